// Discrete adjoint of one ADER-DG step (device), transposing every stage of
// k_predict + k_volume / k_face_flux / k_lift_update:  given U^n and lambda^{n+1} = dJ/dU^{n+1}
// it returns lambda^n = dJ/dU^n and accumulates dJ/dmu0, dJ/dC_d per element.
//
//   k_predict (forward, recomputed)         ->  time-point states U_z of all elements
//   k_adj_face   one wavefront per face: traces of U_z and of lambda on both
//                sides, cotangent of the single-valued flux from both sides'
//                updates, flux VJP for both traces -> trace cotangents per face
//   k_adj_lift   one wavefront per element: transposed lift of its four faces'
//                trace cotangents -> face part of dJ/dU_z
//   k_adj_volume one wavefront per element: predictor restored or recomputed;
//                volume / source VJP at every (z, q); transposed nodal
//                evaluation; Taylor and CK recursion reversed;
//                cell-averaged-tangent VJP (second derivatives of the stress);
//                identity path -> lambda^n
// Every wavefront writes only its own outputs (no atomics).
#pragma once
#include "adjoint_point.hpp"
#include "kernels.hpp"

namespace dgd {

template <int P> struct AdjArgs {
  using T = typename Prec<P>::T;
  using AF = typename Prec<P>::AF;
  StepArgs<P> s;          // forward data (U^n in s.U9 / s.Ua, time points in s.Uz)
  const T* lam;           // [E][KPL][16] lambda^{n+1}
  T* lamOut;              // [E][KPL][16] lambda^n
  T* gtr;                 // [face][side][Nt][Ns][10] cotangents of the face traces
  T* lzf;                 // [E][Nt][KPL][16] their transposed lift (face part of dJ/dU_z)
  double* gmuf;           // [face][side] face part of dJ/dmu0
  const int* fmap;        // [E][4] face * 2 + side
  const AF* VTpk;         // V^T per chunk        (L x 64)
  const AF* STpk;         // Sw^e^T per e, chunk  (64 x L)
  const AF* PTpk;         // Pw^T per chunk       (64 x L)
  const AF* KTpk;         // K^e^T per e          (L x L)
  const double* wq;       // [Q] volume weights
  const double* beta;     // [Ns] face weights
  const T* Dkept;         // [E][N][KPL][16] predictor derivatives of this step (or null)
  const T* Akept;         // [E][48] cell-averaged tangents of this step (or null)
  double* gmu;            // [E] dJ/dmu0 (accumulated)
  double* gcd;            // [E] dJ/dC_d (accumulated)
};

// One wavefront per face (the face list of k_face_flux): traces of U_z and of
// lambda^{n+1} on both sides at the shared face points.  The face flux F* is
// single valued: the first side's update uses -dt|S|/|J| F*, the second side's
// +dt|S'|/|J'| F*, so its cotangent at a point is
// w = gamma_z (-s Lambda- + s' Lambda+).  The flux VJP gives the cotangents of
// both traces, written to gtr[face][side][z][Ns][10] (lifted by k_adj_volume),
// and of both sides' mu0, summed over the face points with their weights into
// gmuf[face][side].
// FP64 below degree 4: two wavefronts per SIMD at the price of a few spilled
// registers (the unconstrained form needs more than one wavefront's share of
// the register file); FP32: at least two, which its registers fit without
// spilling (forcing four spills far more).
template <int N, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P != PREC_F64 || N <= 3 ? 2 : 1)))
void k_adj_face(AdjArgs<P> A, const int* faces, long long nfaces) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  const StepArgs<P>& a = A.s;
  constexpr int L = DM::L, Ns = DM::Ns, Nt = DM::Nt, NST = DM::NST;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  constexpr int R = 11;   // traces keep the 10 quantities (odd stride: no bank conflicts)
  constexpr int TS = NST * 16 * R;
  __shared__ T sTm[Nt * TS];
  __shared__ T sTp[Nt * TS];
  __shared__ T sLm[TS];
  __shared__ T sLp[TS];

  const int lane = threadIdx.x;
  const long long fid = elem_of_block(nfaces);
  if (fid >= nfaces) return;
  const int ef = faces[fid * 2], of = faces[fid * 2 + 1];
  const long long e = ef >> 2;
  const int f = ef & 3;
  const int w = a.conn[ef * 2 + 1];
  const int kind = conn_kind(w), sp = conn_perm(w);
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  // both sides' traces in one pass (a boundary face evaluates its own side
  // twice and uses the first), so that all their loads are in flight together
  const bool inner = kind == 0;
  const long long nb = inner ? (long long)(of >> 2) : e;
  const int nf = inner ? (of & 3) : f;
  const typename PR::AF* Fe = a.Fpk + (size_t)(f * 6 + sp) * NST * KSL * 64;
  const typename PR::AF* Fn =
      a.Fpk + (size_t)(nf * 6 + (inner ? conn_nperm(w) : sp)) * NST * KSL * 64;
  const T* Uze = a.Uz + (size_t)e * DM::UZE;
  const T* Uzn = a.Uz + (size_t)nb * DM::UZE;
  if constexpr (FaceSharedA<P>::value) {
    // the time-point states ([L][10]) one side after the other, all time
    // points together: each trace-matrix fragment is loaded once per side
    Acc Cz[Nt][NST];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int z = 0; z < Nt; ++z) zero_C<P, NST>(Cz[z]);
      wave_gemm_shared_a<P, NST, KSL, Nt, 10, DM::UZT>(side ? Fn : Fe, side ? Uzn : Uze, Cz, lane);
#pragma unroll
      for (int z = 0; z < Nt; ++z)
        store_C<P, NST, R, 10>(Cz[z], (side ? sTp : sTm) + z * TS, Ns, T(1), lane);
    }
  }
#pragma unroll
  for (int z = FaceSharedA<P>::value ? Nt : 0; z <= Nt; ++z) {
    // z < Nt: time-point states ([L][10]); z = Nt: lambda^{n+1} ([KPL][16])
    Acc C[NST], Cn[NST];
    zero_C<P, NST>(C);
    zero_C<P, NST>(Cn);
    if (z < Nt) {
      wave_gemm<P, NST, KSL, 10, KSL, 16, false>(Fe, Uze + z * DM::UZT, C, lane);
      wave_gemm<P, NST, KSL, 10, KSL, 16, false>(Fn, Uzn + z * DM::UZT, Cn, lane);
    } else {
      wave_gemm<P, NST, KSL, 16, KSL, 16, false>(Fe, A.lam + (size_t)e * KPL * 16, C, lane);
      wave_gemm<P, NST, KSL, 16, KSL, 16, false>(Fn, A.lam + (size_t)nb * KPL * 16, Cn, lane);
    }
    store_C<P, NST, R, 10>(C, z < Nt ? sTm + z * TS : sLm, Ns, T(1), lane);
    store_C<P, NST, R, 10>(Cn, z < Nt ? sTp + z * TS : sLp, Ns, T(1), lane);
  }
  __syncthreads();
  T n[3];
  n[0] = (T)a.fgeo[(e * 4 + f) * 4 + 0];
  n[1] = (T)a.fgeo[(e * 4 + f) * 4 + 1];
  n[2] = (T)a.fgeo[(e * 4 + f) * 4 + 2];
  const T se = (T)(a.fgeo[(e * 4 + f) * 4 + 3] * a.dt);
  const T sn = kind == 0 ? (T)(a.fgeo[(nb * 4 + nf) * 4 + 3] * a.dt) : T(0);
  const MatP<T> mp = kind == 0 ? load_mat<T>(a.mat + nb * 8) : m;
  T gmum = T(0), gmup = T(0);
  T* g0 = A.gtr + (size_t)fid * 2 * Nt * Ns * 10;
  T* g1 = g0 + Nt * Ns * 10;
  for (int idx = lane; idx < Ns * Nt; idx += 64) {
    const int z = idx / Ns, i = idx - z * Ns;
    T uM[10], wv[10], gm[10], gp[10];
    const T g = a.gamma[z];
    const T bi = (T)A.beta[i];
    T cm = T(0), cp = T(0);
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      uM[k] = sTm[z * TS + i * R + k];
      gm[k] = T(0);
      gp[k] = T(0);
    }
    if (kind == 0) {
      T uP[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        uP[k] = sTp[z * TS + i * R + k];
        wv[k] = g * (-se * sLm[i * R + k] + sn * sLp[i * R + k]);
      }
      llf_vjp_both(uM, uP, n, m, mp, law, wv, gm, gp, cm, cp);
    } else {
#pragma unroll
      for (int k = 0; k < 10; ++k) wv[k] = g * (-se * sLm[i * R + k]);
      boundary_vjp(kind, uM, n, m, law, wv, gm, cm);
    }
    // the state cotangents take the face weight through the lift; the
    // material cotangents take it here
    gmum += bi * cm;
    gmup += bi * cp;
#pragma unroll
    for (int k = 0; k < 10; ++k) g0[(z * Ns + i) * 10 + k] = gm[k];
    if (kind == 0) {
#pragma unroll
      for (int k = 0; k < 10; ++k) g1[(z * Ns + i) * 10 + k] = gp[k];
    }
  }
  const T s0 = wave_sum(gmum), s1 = wave_sum(gmup);
  if (lane == 0) {
    A.gmuf[fid * 2] = (double)s0;
    A.gmuf[fid * 2 + 1] = (double)s1;
  }
}

// One wavefront per element: the transposed lift of its four faces' trace
// cotangents (the second side's negation is already in them), per time point
// -> lzf[e][z] in the [l][16] layout.
template <int N, int P>
__global__ __launch_bounds__(64) void k_adj_lift(AdjArgs<P> A) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  const StepArgs<P>& a = A.s;
  constexpr int L = DM::L, Ns = DM::Ns, Nt = DM::Nt, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS);
  constexpr int KPN = round_up(Ns, KS), KSN = KPN / KS;
  constexpr int R = Lds<T>::RS;
  constexpr int GB = KPN * R;                      // one time point's cotangents, [Ns][R]
  __shared__ T sG[Nt * GB];

  const int lane = threadIdx.x;
  const long long e = elem_of_block(a.E);
  if (e >= a.E) return;
  for (int i = lane; i < Nt * GB; i += 64) sG[i] = T(0);
  Acc Cz[Nt][MT];
#pragma unroll
  for (int z = 0; z < Nt; ++z) zero_C<P, MT>(Cz[z]);
  // the next face's cotangents are loaded while this face's are lifted
  constexpr int GPL = (Nt * Ns * 10 + 63) / 64;
  T gv[GPL];
  auto load_face = [&](int f) {
    const int fm = A.fmap[e * 4 + f];
    const T* g = A.gtr + ((size_t)(fm >> 1) * 2 + (fm & 1)) * Nt * Ns * 10;
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
      const int idx = lane + 64 * j;
      gv[j] = idx < Nt * Ns * 10 ? g[idx] : T(0);
    }
  };
  load_face(0);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int sp = conn_perm(a.conn[(e * 4 + f) * 2 + 1]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
      const int idx = lane + 64 * j;
      if (idx < Nt * Ns * 10) {
        const int zi = idx / 10, k = idx - zi * 10, z = zi / Ns, i = zi - z * Ns;
        sG[z * GB + i * R + k] = gv[j];
      }
    }
    if (f < 3) load_face(f + 1);
    __syncthreads();
    // one lift matrix for all time points: each of its fragments is loaded once
    wave_gemm_shared_a<P, MT, KSN, Nt, R, GB>(a.Lpk + (size_t)(f * 6 + sp) * MT * KSN * 64, sG, Cz,
                                             lane);
  }
#pragma unroll
  for (int z = 0; z < Nt; ++z)
    store_C<P, MT, 16>(Cz[z], A.lzf + ((size_t)e * Nt + z) * KPL * 16, KPL, T(1), lane);
}

// At degree 4 the adjoint of the volume terms runs as two launches, each with
// its own register and LDS budget (one launch holds more than a SIMD's
// registers): k_adj_points (the volume and source cotangents at the time
// points, dJ/dU_z to HBM), then k_adj_volume<N, P, false> (the predictor
// reversed).  Below degree 4 k_adj_volume<N, P, true> does both.
template <int N> struct AdjSplit {
  static constexpr bool value = N >= 4;
};

// LDS of k_adj_points: lambda^{n+1}, then the time-point state being
// evaluated (then its cotangent); the point values / integrands of a chunk;
// the per-point cotangents that lambda^{n+1} gives.
template <int N, int P> struct AdjPtLDS {
  using T = typename Prec<P>::T;
  static constexpr int KPL = round_up(Dims<N>::L, Prec<P>::KS);
  static constexpr int R = Lds<T>::RS;
  union {
    T Lam[KPL * 16];
    T Z[KPL * 16];              // lambda^{n+1} is spent before the first time point
  };
  T X[64 * R];
  T Lp[Dims<N>::NCH][10][64];   // per point: velocity, stress and rate cotangents
};

// One wavefront per element: the volume and source terms transposed.
// dJ/dG^e at the volume points is dt Sw^e^T lambda, folded at once into the
// cotangents of the velocity and of the stress per point and unit time weight
// (the flux is linear in both), and dJ/dr is dt Pw^T lambda_alpha; at every
// (z, q) the pointwise VJP of sigma and r_alpha at the time-point state U_z
// (read from HBM, where k_predict left it) and the transposed nodal
// evaluation give the volume part of dJ/dU_z, which joins the face part in
// lzf[e][z]; the material cotangents of the volume points join gmu, gcd.
template <int N, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P == PREC_F64 ? 2 : 4)))
void k_adj_points(AdjArgs<P> A) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  const StepArgs<P>& a = A.s;
  constexpr int L = DM::L, Q = DM::Q, Nt = DM::Nt, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS, KSQ = 64 / KS;
  constexpr int DS = 16, DPL = KPL * DS / 64;
  using SL = AdjPtLDS<N, P>;
  constexpr int R = SL::R;
  __shared__ SL S;
  T* const sX = S.X;
  T* const sZ = S.Z;
  const int lane = threadIdx.x;
  const long long e = elem_of_block(a.E);
  if (e >= a.E) return;
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  T Ji[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ji[k] = (T)a.geo[e * 16 + k];
  const T ir = T(1) / m.rho;
  for (int i = lane; i < KPL * DS; i += 64) S.Lam[i] = A.lam[(size_t)e * KPL * 16 + i];
  T gmu = T(0), gcd = T(0);
  __syncthreads();

  // per point and unit time weight: Lp[c][k][lane], k = 0..2 velocity,
  // 3..8 stress, 9 damage rate
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    T LV[3], LS[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) LV[k] = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) LS[k] = T(0);
#pragma unroll 1
    for (int ee = 0; ee < 3; ++ee) {
      Acc C[4];
      zero_C<P, 4>(C);
      wave_gemm<P, 4, KSL, DS>(A.STpk + (size_t)(ee * NCH + c) * 4 * KSL * 64, S.Lam, C, lane);
      store_C<P, 4>(C, sX, 64, (T)a.dt, lane);
      __syncthreads();
      // G^e_(ij) = -(J_ej v_i + J_ei v_j)/2,  G^e_(v_i) = -(1/rho) sum_d J_ed sigma_id
      T Jr[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) Jr[d] = ee == 0 ? Ji[d] : (ee == 1 ? Ji[3 + d] : Ji[6 + d]);
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int ii = kVI[p], jj = kVJ[p];
        const T lg = sX[lane * R + p];
        LV[ii] += T(-0.5) * Jr[jj] * lg;
        LV[jj] += T(-0.5) * Jr[ii] * lg;
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const T lg = sX[lane * R + 6 + ii] * (-ir);
#pragma unroll
        for (int d = 0; d < 3; ++d) LS[sym_idx(ii, d)] += lg * Jr[d];
      }
      __syncthreads();
    }
    Acc C[4];
    zero_C<P, 4>(C);
    wave_gemm<P, 4, KSL, DS>(A.PTpk + (size_t)c * 4 * KSL * 64, S.Lam, C, lane);
    store_C<P, 4>(C, sX, 64, (T)a.dt, lane);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) S.Lp[c][k][lane] = LV[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) S.Lp[c][3 + k][lane] = LS[k];
    S.Lp[c][9][lane] = sX[lane * R + 9];
    __syncthreads();
  }

  const T* Uze = a.Uz + (size_t)e * DM::UZE;
#pragma unroll 1
  for (int z = 0; z < Nt; ++z) {
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
      sZ[idx] = (l < L && p < 10) ? Uze[z * DM::UZT + l * 10 + p] : T(0);
    }
    __syncthreads();
    const T g = a.gamma[z];
    Acc Cl[MT];
    zero_C<P, MT>(Cl);
#pragma unroll 1
    for (int c = 0; c < NCH; ++c) {
      Acc C[4];
      zero_C<P, 4>(C);
      wave_gemm_tiles<P, 4, KSL, DS>(a.Vpk + (size_t)c * 4 * KSL * 64, sZ, C, lane);
      store_C<P, 4>(C, sX, 64, T(1), lane);
      __syncthreads();
      const int q = 64 * c + lane;
      T gu[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) gu[k] = T(0);
      if (q < Q) {
        T u[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
        T ls[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) ls[k] = g * S.Lp[c][3 + k][lane];
#pragma unroll
        for (int k = 0; k < 3; ++k) gu[6 + k] += g * S.Lp[c][k][lane];
        const Parts<T> pp = cdm_parts(u, law);
        stress_vjp_p(pp, u, m, ls, gu, gmu);
        rate_vjp_p(pp, u, m, g * S.Lp[c][9][lane], gu, gcd);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) sX[lane * R + k] = k < 10 ? gu[k] : T(0);
      __syncthreads();
      wave_gemm_tiles<P, MT, KSQ>(A.VTpk + (size_t)c * MT * KSQ * 64, sX, Cl, lane);
      __syncthreads();
    }
    // the time-point state is spent: the volume part of dJ/dU_z goes there,
    // then joins the face part
    store_C<P, MT, DS>(Cl, sZ, KPL, T(1), lane);
    __syncthreads();
    T* lz = A.lzf + ((size_t)e * Nt + z) * KPL * 16;
#pragma unroll
    for (int j = 0; j < DPL; ++j) lz[lane + 64 * j] += sZ[lane + 64 * j];
    __syncthreads();
  }
  const T gm = wave_sum(gmu), gc = wave_sum(gcd);
  if (lane == 0) {
    A.gmu[e] += (double)gm;
    A.gcd[e] += (double)gc;
  }
}

// Derivatives D^i of the predictor in registers (one LDS buffer, which also
// takes the time-point states), or all of them in LDS: as in the forward
// kernel, except FP64, whose adjoint registers would not fit, and the fused
// degree-4 form.
template <int N, int P> struct AdjRegs {
  static constexpr bool value = P != PREC_F64 && (N <= 3 || AdjSplit<N>::value);
  static constexpr int ND = value ? 1 : N + 1;
};

// PTS: this launch also transposes the volume and source terms at the time
// points (else k_adj_points has, and lzf holds all of dJ/dU_z).
template <int N, int P, bool PTS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(AdjRegs<N, P>::value ? (PTS ? 3 : 2) : 1)))
void k_adj_volume(AdjArgs<P> A) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  const StepArgs<P>& a = A.s;
  constexpr int L = DM::L, Q = DM::Q, Nt = DM::Nt, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS, KSQ = 64 / KS;
  constexpr bool REGS = AdjRegs<N, P>::value;
  constexpr int ND = AdjRegs<N, P>::ND;
  // with the derivatives in registers the time-point buffer W is unused, and
  // the right-hand sides Y_e and their cotangents keep 10 columns and one
  // zero column (row stride RB = 11), as do the cotangents dJ/dD^i (row
  // stride RL); else both keep 16 columns
  constexpr int AWM = REGS ? 2 : 0;
  using SL = PredLDS<N, P, ND, AWM>;
  constexpr int R = SL::R, RB = SL::RB, DS = SL::DS, DPL = SL::DPL;
  constexpr int NCB = RB == R ? 16 : 10;
  constexpr int RL = REGS ? 11 : DS, NCL = REGS ? 10 : 16;
  static_assert(DS == 16, "adjoint states are exchanged with HBM row by row");
  __shared__ SL S;
  // sLD[i] = dJ/dD^i; sLD[0] starts as lambda^{n+1} (the identity path) and
  // ends as lambda^n minus the nodal path of the tangent and source at t_n
  __shared__ T sLD[N + 1][KPL * RL];
  // position in sLD of entry idx of a [KPL][16] matrix (-1: a column not kept)
  auto lpos = [&](int idx) -> int {
    const int l = idx >> 4, p = idx & 15;
    return (RL == 16 || p < 10) ? l * RL + p : -1;
  };
  T dreg[REGS ? (N + 1) * DPL : 1];
  T* const sX = S.B;
  T* const sLam = sLD[0];
  T* const sLA = S.B;     // dJ/dA*_e, between the CK reversal and the t_n pass
  T* const sLds = S.Acc;  // its cell-average cotangent (the average itself is spent)
  // time-point state, then dJ/dU_z; at the end the nodal path at t_n
  T* const sZ = [&]() -> T* {
    if constexpr (REGS)
      return S.D[0];
    else
      return S.W;
  }();
  const int lane = threadIdx.x;
  // D^i[idx] for idx = lane + 64 j
  auto Dv = [&](int i, int j) -> T {
    if constexpr (REGS)
      return dreg[i * DPL + j];
    else
      return S.D[i][lane + 64 * j];
  };
  // D^i to the LDS buffer read by the matrix cores (a no-op when all are there)
  auto Dlds = [&](int i) -> const T* {
    if constexpr (REGS) {
#pragma unroll
      for (int j = 0; j < DPL; ++j) S.D[0][lane + 64 * j] = dreg[i * DPL + j];
      return S.D[0];
    } else {
      return S.D[i];
    }
  };

  const long long e = elem_of_block(a.E);
  if (e >= a.E) return;
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  if (A.Dkept)
    predictor_restore<N, P, ND, REGS>(a, e, S, m, A.Dkept, A.Akept, lane, dreg);
  else
    predictor_stage<N, P, ND, REGS, AWM>(a, e, S, m, lane, dreg);
  for (int i = lane; i < (N + 1) * KPL * RL; i += 64) (&sLD[0][0])[i] = T(0);
  __syncthreads();
  for (int idx = lane; idx < KPL * DS; idx += 64) {
    const int o = lpos(idx);
    if (o >= 0) sLam[o] = A.lam[(size_t)e * KPL * 16 + idx];
  }
  T Ji[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ji[k] = S.J[k];
  const T ir = T(1) / m.rho;
  T gmu = T(0), gcd = T(0);
  __syncthreads();

  if constexpr (!PTS) {
    // dJ/dU_z complete in lzf: the Taylor series reversed,
    // dJ/dD^i += (tau_z dt)^i / i! dJ/dU_z
    for (int z = 0; z < Nt; ++z) {
      T cz[N + 1];
      cz[0] = T(1);
      const T h = a.tau[z] * (T)a.dt;
#pragma unroll
      for (int i = 1; i <= N; ++i) cz[i] = cz[i - 1] * h / T(i);
      const T* lz = A.lzf + ((size_t)e * Nt + z) * KPL * 16;
      for (int idx = lane; idx < KPL * DS; idx += 64) {
        const int o = lpos(idx);
        if (o < 0) continue;
        const T v = lz[idx];
#pragma unroll
        for (int i = 0; i <= N; ++i) sLD[i][o] += cz[i] * v;
      }
    }
    __syncthreads();
  } else {
  // dJ/dG^e at the volume points: dt Sw^e^T lambda, folded at once into the
  // cotangents of the velocity (LV) and of the stress (LS) at each point, per
  // unit time weight (the flux is linear in both);  dJ/dr: dt Pw^T lambda_alpha
  T LV[NCH][3], LS[NCH][6];
  T Ls[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
#pragma unroll
    for (int k = 0; k < 3; ++k) LV[c][k] = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) LS[c][k] = T(0);
#pragma unroll
    for (int ee = 0; ee < 3; ++ee) {
      Acc C[4];
      zero_C<P, 4>(C);
      wave_gemm<P, 4, KSL, RL, KSL, NCL>(A.STpk + (size_t)(ee * NCH + c) * 4 * KSL * 64, sLam, C,
                                         lane);
      store_C<P, 4>(C, sX, 64, (T)a.dt, lane);
      __syncthreads();
      // G^e_(ij) = -(J_ej v_i + J_ei v_j)/2,  G^e_(v_i) = -(1/rho) sum_d J_ed sigma_id
      const T* Jr = Ji + ee * 3;
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int ii = kVI[p], jj = kVJ[p];
        const T lg = sX[lane * R + p];
        LV[c][ii] += T(-0.5) * Jr[jj] * lg;
        LV[c][jj] += T(-0.5) * Jr[ii] * lg;
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const T lg = sX[lane * R + 6 + ii] * (-ir);
#pragma unroll
        for (int d = 0; d < 3; ++d) LS[c][sym_idx(ii, d)] += lg * Jr[d];
      }
      __syncthreads();
    }
    Acc C[4];
    zero_C<P, 4>(C);
    wave_gemm<P, 4, KSL, RL, KSL, NCL>(A.PTpk + (size_t)c * 4 * KSL * 64, sLam, C, lane);
    store_C<P, 4>(C, sX, 64, (T)a.dt, lane);
    __syncthreads();
    Ls[c] = sX[lane * R + 9];
    __syncthreads();
  }

  // volume and source cotangents at every time point -> dJ/dU_z, and the
  // Taylor series reversed on the way: dJ/dD^i += (tau_z dt)^i / i! dJ/dU_z
  for (int z = 0; z < Nt; ++z) {
    T cz[N + 1];
    cz[0] = T(1);
    const T h = a.tau[z] * (T)a.dt;
#pragma unroll
    for (int i = 1; i <= N; ++i) cz[i] = cz[i - 1] * h / T(i);
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      T v = T(0);
#pragma unroll
      for (int i = 0; i <= N; ++i) v += cz[i] * Dv(i, j);
      sZ[lane + 64 * j] = v;
    }
    __syncthreads();
    const T g = a.gamma[z];
    Acc Cl[MT];
    zero_C<P, MT>(Cl);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      Acc C[4];
      zero_C<P, 4>(C);
      wave_gemm<P, 4, KSL, DS>(a.Vpk + (size_t)c * 4 * KSL * 64, sZ, C, lane);
      store_C<P, 4>(C, sX, 64, T(1), lane);
      __syncthreads();
      const int q = 64 * c + lane;
      T gu[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) gu[k] = T(0);
      if (q < Q) {
        T u[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
        T ls[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) ls[k] = g * LS[c][k];
#pragma unroll
        for (int k = 0; k < 3; ++k) gu[6 + k] += g * LV[c][k];
        const Parts<T> pp = cdm_parts(u, law);
        stress_vjp_p(pp, u, m, ls, gu, gmu);
        rate_vjp_p(pp, u, m, g * Ls[c], gu, gcd);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) sX[lane * R + k] = k < 10 ? gu[k] : T(0);
      __syncthreads();
      wave_gemm<P, MT, KSQ>(A.VTpk + (size_t)c * MT * KSQ * 64, sX, Cl, lane);
      __syncthreads();
    }
    // the time-point state is spent: dJ/dU_z goes there
    store_C<P, MT, DS>(Cl, sZ, KPL, T(1), lane);
    __syncthreads();
    const T* lz = A.lzf + ((size_t)e * Nt + z) * KPL * 16;
    for (int idx = lane; idx < KPL * DS; idx += 64) {
      const int o = lpos(idx);
      if (o < 0) continue;
      const T v = sZ[idx] + lz[idx];
#pragma unroll
      for (int i = 0; i <= N; ++i) sLD[i][o] += cz[i] * v;
    }
    __syncthreads();
  }
  }

  // Cauchy-Kovalevskaya recursion reversed: D^i = -sum_e K^e D^{i-1} A*_e^T (+ source).
  // All three contractions on the matrix cores; dJ/dA*_e stays in registers.
  for (int i = lane; i < 3 * KPL * RB; i += 64) S.B[i] = T(0);   // padding rows of dJ/dY_e
  Acc CA[3];
  zero_C<P, 3>(CA);
  __syncthreads();
#pragma unroll
  for (int i = N; i >= 1; --i) {
    const T* Dm = Dlds(i - 1);
#pragma unroll
    for (int ee = 0; ee < 3; ++ee) {
      Acc C[MT];
      zero_C<P, MT>(C);
      wave_gemm<P, MT, KSL, RL, KSL, NCL>(A.KTpk + (size_t)ee * MT * KSL * 64, sLD[i], C, lane);
      store_C<P, MT, RB, NCB>(C, S.B + ee * KPL * RB, L, T(-1), lane);   // dJ/dY_e = -K^e^T dJ/dD^i
    }
    __syncthreads();
    // dJ/dA*_e[p][q] += sum_l dJ/dY_e[l][p] D^{i-1}[l][q]   (A = dJ/dY_e^T from LDS)
#pragma unroll
    for (int ee = 0; ee < 3; ++ee)
#pragma unroll
      for (int st = 0; st < KSL; ++st) {
        const T av = S.B[(ee * KPL + KS * st + (lane >> 4)) * RB + bcol<NCB>(lane)];
        CA[ee] = PR::mma(av, PR::template loadB<DS>(Dm, st, lane), CA[ee]);
      }
    // dJ/dD^{i-1}[l][q] += sum_e sum_p dJ/dY_e[l][p] A*_e[p][q]   (K = p, 3 steps)
    {
      Acc CD[MT];
      zero_C<P, MT>(CD);
      const int col = lane & 15;
#pragma unroll
      for (int ee = 0; ee < 3; ++ee)
#pragma unroll
        for (int st = 0; st < 3; ++st) {
          const int k = KS * st + (lane >> 4);
          const T bv = (k < 10 && col < 10) ? S.A[ee * 100 + k * 10 + col] : T(0);
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            const int row = 16 * t + col;
            const T av = (row < L && k < 10) ? S.B[(ee * KPL + row) * RB + k] : T(0);
            CD[t] = PR::mma(av, bv, CD[t]);
          }
        }
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) {
          const int r = 16 * t + PR::crow(lane, i4);
          if (r < L && col < NCL) sLD[i - 1][r * RL + col] += CD[t][i4];
        }
    }
    __syncthreads();
  }
  // damage source at t_n: dJ/dr_q = (Pw^T dJ/dD^1)_q in column 9
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    Acc C[4];
    zero_C<P, 4>(C);
    wave_gemm<P, 4, KSL, RL, KSL, NCL>(A.PTpk + (size_t)c * 4 * KSL * 64, sLD[1], C, lane);
    store_C<P, 4>(C, sX, 64, T(1), lane);
    __syncthreads();
    S.R_[64 * c + lane] = sX[lane * R + 9];
    __syncthreads();
  }
  // dJ/dA*_e from the accumulators (S.B is free again)
#pragma unroll
  for (int ee = 0; ee < 3; ++ee)
#pragma unroll
    for (int i4 = 0; i4 < 4; ++i4) {
      const int r = PR::crow(lane, i4), c = lane & 15;
      if (r < 10 && c < 10) sLA[ee * 100 + r * 10 + c] = CA[ee][i4];
    }
  __syncthreads();
  // dJ/dBbar through A*_e[6+i][q] = -(1/rho) sum_d Theta^-1_ed dsbar[sym(i,d)][col(q)]
  if (lane < 42) {
    const int k = lane / 7, c = lane % 7, q = c < 6 ? c : 9;
    T s = T(0);
#pragma unroll
    for (int ee = 0; ee < 3; ++ee)
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (sym_idx(ii, d) == k) s += -ir * Ji[ee * 3 + d] * sLA[ee * 100 + (6 + ii) * 10 + q];
    sLds[lane] = s;
  }
  __syncthreads();
  // mu0 enters the tangent as 2 mu0 on the strain diagonal (the average keeps it)
  if (lane == 0) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) s += T(2) * sLds[k * 7 + k];
    gmu += s;
  }
  // pointwise tangent and source cotangents at t_n -> dJ/dU^n (nodal path)
  T lt[6][7];
  Acc Cu[MT];
  zero_C<P, MT>(Cu);
  const T* D0 = Dlds(0);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    Acc C[4];
    zero_C<P, 4>(C);
    wave_gemm<P, 4, KSL, DS>(a.Vpk + (size_t)c * 4 * KSL * 64, D0, C, lane);
    store_C<P, 4>(C, sX, 64, T(1), lane);
    __syncthreads();
    const int q = 64 * c + lane;
    T gu[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) gu[k] = T(0);
    if (q < Q) {
      T u[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
      const T wgt = (T)A.wq[q] * a.inv_wsum;
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int j = 0; j < 7; ++j) lt[k][j] = wgt * sLds[k * 7 + j];
      const Parts<T> pp = cdm_parts(u, law);
      tangent_vjp_p(pp, u, m, lt, gu);
      rate_vjp_p(pp, u, m, S.R_[q], gu, gcd);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) sX[lane * R + k] = k < 10 ? gu[k] : T(0);
    __syncthreads();
    wave_gemm<P, MT, KSQ>(A.VTpk + (size_t)c * MT * KSQ * 64, sX, Cu, lane);
    __syncthreads();
  }
  store_C<P, MT, DS>(Cu, sZ, KPL, T(1), lane);
  __syncthreads();
  // lambda^n = (lambda^{n+1} + dJ/dD^0, held in sLD[0]) + nodal path
  T* out = A.lamOut + (size_t)e * KPL * 16;
  for (int idx = lane; idx < KPL * DS; idx += 64) {
    const int o = lpos(idx);
    out[idx] = (o >= 0 ? sLD[0][o] : T(0)) + sZ[idx];
  }
  const T gm = wave_sum(gmu), gc = wave_sum(gcd);
  if (lane == 0) {
    double gf = 0.0;
    for (int f = 0; f < 4; ++f) {
      const int fm = A.fmap[e * 4 + f];
      gf += A.gmuf[(size_t)(fm >> 1) * 2 + (fm & 1)];
    }
    A.gmu[e] += (double)gm + gf;
    A.gcd[e] += (double)gc;
  }
}

// receiver misfit: lambda[e_r][l][6+c] += dL/dv_rc phi_l(xi_r)
template <class T>
__global__ void k_adj_receivers(int nrec, int L, int kpl, const long long* elem, const double* phi,
                                const double* dldv, T* lam) {
  const int idx = threadIdx.x;   // (c, l)
  if (idx >= 3 * L) return;
  const int c = idx / L, l = idx % L;
  for (int r = 0; r < nrec; ++r) {
    T* dst = lam + ((size_t)elem[r] * kpl + l) * 16 + 6 + c;
    *dst = (T)((double)*dst + dldv[r * 3 + c] * phi[r * L + l]);
  }
}

// layout conversions of the adjoint state: [E][10][L] FP64 <-> [E][KPL][16]
template <class T>
__global__ void k_lam_from_f64(long long E, int L, int kpl, const double* in, T* lam) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * kpl * 16) return;
  const long long e = idx / (kpl * 16);
  const int r = (int)(idx % (kpl * 16)), l = r / 16, p = r % 16;
  lam[idx] = (l < L && p < 10) ? (T)in[(e * 10 + p) * L + l] : T(0);
}

template <class T>
__global__ void k_lam_to_f64(long long E, int L, int kpl, const T* lam, double* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * 10 * L) return;
  const long long e = idx / (10 * L);
  const int p = (int)((idx / L) % 10), l = (int)(idx % L);
  out[idx] = (double)lam[(e * kpl + l) * 16 + p];
}

}  // namespace dgd
