// Per-step kernels of the ADER-DG update (gfx950).  One 64-lane wavefront owns
// one tetrahedron; workgroups are mapped to elements so that each of the eight
// XCDs walks a contiguous range of elements (neighbours share an L2).
//
// k_predict  (paper Appendix A.1)
//   nodal values at t_n -> pointwise CDM tangent -> cell-averaged Jacobians
//   A*_e = sum_d Theta^-1_ed Bbar^d  (Eq. CKIter-ref)
//   D^i = -sum_e K^e D^{i-1} A*_e^T, + nodal damage source at i = 1
//   (Eqs. CKIter-ref-matrix, CKIter-ref-source)
//   time points U_z = sum_i (tau_z dt)^i/i! D^i  (Eq. taylor_expansion) -> HBM
// k_volume  (the volume/source terms of Appendix A.2)
//   volume term dt sum_z gamma_z sum_e Sw^e F^e(U_z) and damage source
//   (Eqs. 3rd term, rhs term; the nodal projection followed by the stiffness
//   equals quadrature with Sw = w_q dphi/dxi), partial update written out.
// k_face_flux  (Appendix A.2 Eq. 2nd term, A.3), one wavefront per face
//   traces of both sides at the shared face points for every time point,
//   LLF (or boundary) flux, time quadrature -> [face][Ns][10] in HBM.
// k_lift_update  lift of the four face fluxes of an element, final update.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.hpp"
#include "physics.hpp"

namespace dgd {

template <int N> struct Dims {
  static constexpr int L = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Q = (N + 1) * (N + 1) * (N + 1);
  static constexpr int Ns = (N + 1) * (N + 1);
  static constexpr int Nt = N + 1;
  static constexpr int NCH = (Q + 63) / 64;  // 64-point chunks of volume points
  static constexpr int MT = (L + 15) / 16;   // 16-row tiles of a mode-indexed output
  static constexpr int NST = (Ns + 15) / 16; // 16-row tiles of a face-point output
  // time-point states in HBM, [E][Nt][L][10]: UZT values per time point,
  // UZE per element (see StepArgs::Uz)
  static constexpr int UZT = L * 10;
  static constexpr int UZE = Nt * UZT;
};

// connectivity word: bits 0-1 face kind (0 interior, 1 free, 2 absorbing),
// 2-4 own point permutation, 5-6 neighbour face, 7-9 neighbour permutation
__host__ __device__ inline int conn_kind(int w) { return w & 3; }
__host__ __device__ inline int conn_perm(int w) { return (w >> 2) & 7; }
__host__ __device__ inline int conn_nface(int w) { return (w >> 5) & 3; }
__host__ __device__ inline int conn_nperm(int w) { return (w >> 7) & 7; }

template <int P> struct StepArgs {
  using T = typename Prec<P>::T;
  using AF = typename Prec<P>::AF;
  long long E;
  const T* U9;          // [E][9][L] current wave quantities
  const double* Ua;     // [E][L] current damage (FP64)
  T* W9;                // [E][9][L] next state
  double* Wa;           // [E][L]
  // [E][Nt][L][10] time-point states, no padding.  The matrix cores read them
  // in place as B operands with row stride 10: lanes of columns 10..15 read
  // the next row's first entries and feed only output columns that are
  // dropped, and the k-steps past row L (up to KPL) meet zero columns of the
  // reference matrices; the allocation holds KPL * 16 zeroed entries past the
  // last element so that those reads stay inside it and finite.
  T* Uz;
  const double* geo;    // [E][16]: Theta^-1 (row e, column d), |J|
  const double* fgeo;   // [E][4][4]: outward normal, |S_f|/|J|
  const double* mat;    // [E][8]: rho, lambda0, mu0, gamma_r, xi0, C_d
  const int* conn;      // [E][4][2]: neighbour, connectivity word
  const AF* Vpk;        // volume evaluation, per 64-point chunk
  const AF* Kpk;        // [K^0 K^1 K^2]
  const AF* Spk;        // Sw^e per chunk
  const AF* Fpk;        // face traces [f][perm]
  const AF* Lpk;        // lift [f][perm]
  const typename Prec<Accurate<P>::value>::AF* Ppk;   // w_q phi_l(xi_q) per chunk
  const double* wq;     // [Q] volume quadrature weights
  T* Dkeep;             // [E][N][KPL][16] D^1..D^N kept for the adjoint (or null)
  T* Akeep;             // [E][48] cell-averaged tangent kept for the adjoint (or null)
  double dt;
  T amax, smin, inv_wsum;
  T tau[8], gamma[8];
  int* flag;
  // local time stepping: the elements a launch covers (null: all E), the
  // cluster of every element, the cluster being corrected (-1: global step),
  // flux integrals accumulated for the coarser side of cluster boundaries
  // [face][Ns][10], and where the final update goes (null: W9 / Wa)
  const int* elist;
  long long nlist;
  const signed char* ecl;
  int lts_c;
  T* facc;
  T* O9;
  double* Oa;
};

// element of this workgroup (-1: none), through the element list if any
template <int P>
__device__ inline long long elem_index(const StepArgs<P>& a) {
  const long long n = a.elist ? a.nlist : a.E;
  const long long per = (n + 7) / 8;
  const long long b = blockIdx.x;
  const long long i = (b % 8) * per + b / 8;
  if (i >= n) return -1;
  return a.elist ? (long long)a.elist[i] : i;
}

__device__ inline long long elem_of_block(long long E) {
  const long long per = (E + 7) / 8;
  const long long b = blockIdx.x;
  return (b % 8) * per + b / 8;
}

template <class T>
__device__ inline MatP<T> load_mat(const double* p) {
  MatP<T> m;
  m.rho = (T)p[0];
  m.lam = (T)p[1];
  m.mu = (T)p[2];
  m.gr = (T)p[3];
  m.xi0 = (T)p[4];
  m.cd = (T)p[5];
  return m;
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ constexpr int kVI[6] = {0, 1, 2, 0, 1, 2};
__device__ constexpr int kVJ[6] = {0, 1, 2, 1, 2, 0};

// The time-point buffer W and A*_e: separate (AW = 0), or sharing storage
// (AW = 1: the adjoint's register form, which puts its time-point states
// elsewhere), or no W at all (AW = 2: the forward prediction, which writes its
// time-point states from registers).
template <class T, int NW, int AW> struct PredWA {
  T W[NW];                // time-point state / scratch
  T A[300];               // A*_e (3 x 10 x 10)
};
template <class T, int NW> struct PredWA<T, NW, 1> {
  union {
    T W[NW];
    T A[300];
  };
};
template <class T, int NW> struct PredWA<T, NW, 2> {
  T A[300];
};

// LDS working set of the predictor of one element (one wavefront).  Matrices
// with 16 columns (the 10 quantities, padded) use the row stride R where they
// are read or written one row per lane, 16 elsewhere.
// ND = N + 1 keeps every time derivative in LDS (the adjoint needs them all);
// ND = 1 keeps only the one being formed (it overwrites its predecessor once
// the right-hand sides are built) and leaves a copy of each in registers, DPL
// values per lane, for the Taylor sums.
template <int N, int P, int ND = N + 1, int AW = 0>
struct PredLDS : PredWA<typename Prec<P>::T, round_up(Dims<N>::L, Prec<P>::KS) * 16, AW> {
  using T = typename Prec<P>::T;
  static constexpr int L = Dims<N>::L, NCH = Dims<N>::NCH;
  static constexpr int KPL = round_up(L, Prec<P>::KS);
  static constexpr int R = Lds<T>::RS;   // rows read one per lane
  static constexpr int DS = 16;          // D, W: read linearly and as matrix-core B operands
  static constexpr int DPL = KPL * DS / 64;
  static_assert(KPL * DS % 64 == 0, "derivatives split evenly over the lanes");
  // row stride of the CK right-hand sides Y_e: the forward prediction keeps
  // their 10 quantity columns and one zero column (odd stride; the matrix
  // cores read the zero column for the other 6), the adjoint reuses the
  // buffer with stride R
  static constexpr int RB = AW == 2 ? 11 : R;
  static constexpr int BIG = 64 * R > 3 * KPL * RB ? 64 * R : 3 * KPL * RB;
  T D[ND][KPL * DS];      // time derivatives D^i in buffer i % ND, [l][16] layout
  T B[BIG];               // nodal values, tangent blocks, CK right-hand sides (aliased)
  T R_[NCH * 64];         // nodal damage rate at t_n
  T Acc[48];              // cell-averaged tangent (6 x 7)
  T J[9];                 // Theta^-1
};

// A*_e = sum_d Theta^-1_ed Bbar^d, rows p, columns q (10 x 10 each), from
// Theta^-1 (S.J) and the cell-averaged tangent (S.Acc)
template <int N, int P, int ND, int AW>
__device__ inline void build_Astar(PredLDS<N, P, ND, AW>& S, const MatP<typename Prec<P>::T>& m,
                                   int lane) {
  using T = typename Prec<P>::T;
  for (int i = lane; i < 300; i += 64) {
    const int ee = i / 100, p = (i / 10) % 10, q = i % 10;
    T v = T(0);
    if (p < 6 && q >= 6 && q < 9) {
      const int mm = q - 6, ii = kVI[p], jj = kVJ[p];
      v = T(-0.5) * ((ii == mm ? S.J[ee * 3 + jj] : T(0)) + (jj == mm ? S.J[ee * 3 + ii] : T(0)));
    } else if (p >= 6 && p < 9 && (q < 6 || q == 9)) {
      const int ii = p - 6, col = q < 6 ? q : 6;
      T s = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) s += S.J[ee * 3 + d] * S.Acc[sym_idx(ii, d) * 7 + col];
      v = -s / m.rho;
    }
    S.A[i] = v;
  }
}

// Prediction (Appendix A.1): load U^n, cell-averaged tangent, A*_e, damage
// source at t_n, Cauchy-Kovalevskaya recursion.  Leaves D^0..D^N in S.D
// (REGS false, ND = N + 1; dreg unused and may be null), or in
// dreg[i * DPL + j] = D^i[lane + 64 j] (REGS true, ND = 1).  With AW, S.A is
// not kept past the recursion.
template <int N, int P, int ND, bool REGS, int AW = 0, class LW = CdmLaw>
__device__ inline void predictor_stage(const StepArgs<P>& a, long long e, PredLDS<N, P, ND, AW>& S,
                                       const MatP<typename Prec<P>::T>& m, int lane,
                                       typename Prec<P>::T* dreg) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  constexpr int PA_ = Accurate<P>::value;
  using PA = Prec<PA_>;
  using DM = Dims<N>;
  constexpr int L = DM::L, Q = DM::Q, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  constexpr int KSQA = 64 / PA::KS;
  using SL = PredLDS<N, P, ND, AW>;
  constexpr int R = SL::R, RB = SL::RB, DS = SL::DS, DPL = SL::DPL;
  static_assert(REGS ? ND == 1 : ND == N + 1, "one buffer with register copies, or all");
  T* const sX = S.B;
  const Law<T> law{a.amax, a.smin};

  for (int i = lane; i < ND * KPL * DS; i += 64) (&S.D[0][0])[i] = T(0);
  const T* U9 = a.U9 + e * 9 * L;
  for (int i = lane; i < 10 * L; i += 64) {
    const int p = i / L, l = i - p * L;
    S.D[0][l * DS + p] = p < 9 ? U9[i] : (T)a.Ua[e * L + l];
  }
  if (lane < 9) S.J[lane] = (T)a.geo[e * 16 + lane];
  __syncthreads();
  if constexpr (REGS) {
#pragma unroll
    for (int j = 0; j < DPL; ++j) dreg[j] = S.D[0][lane + 64 * j];
  }

  // cell average of the pointwise tangent, sum_q w_q ds_q / sum_q w_q: the
  // weighted tangents go to LDS 16 entries at a time; lane (c, g) sums column
  // c over the rows 16g..16g+15, the four partial sums meet by lane shuffles.
  // Nodal damage rate at t_n on the way.
  T cav[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    Acc C[4];
    zero_C<P, 4>(C);
    wave_gemm<P, 4, KSL, DS>(a.Vpk + (size_t)c * 4 * KSL * 64, S.D[0], C, lane);
    store_C<P, 4>(C, sX, 64, T(1), lane);
    __syncthreads();
    const int q = 64 * c + lane;
    T ds[6][7];
    T r = T(0);
    if (q < Q) {
      T u[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
      LW::tangent(u, m, law, ds);
      r = -LW::rate(u, m, law);   // negated: it joins the CK contraction stored with -1
      const T wq = (T)a.wq[q];
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int j = 0; j < 7; ++j) ds[k][j] *= wq;
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int j = 0; j < 7; ++j) ds[k][j] = T(0);
    }
    S.R_[q] = r;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * t + jj;
        sX[lane * R + jj] = j < 42 ? ds[j / 7][j % 7] : T(0);
      }
      __syncthreads();
      const int col = lane & 15, g = lane >> 4;
      T sum = T(0);
#pragma unroll
      for (int i = 0; i < 16; ++i) sum += sX[(16 * g + ((i + g) & 15)) * R + col];
      cav[t] += sum;
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    cav[t] += __shfl_xor(cav[t], 16, 64);
    cav[t] += __shfl_xor(cav[t], 32, 64);
  }
  if (lane < 16) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (16 * t + lane < 42) S.Acc[16 * t + lane] = cav[t] * a.inv_wsum;
  }
  __syncthreads();

  build_Astar<N, P>(S, m, lane);
  // The right-hand-side buffer held nodal values before: clear it so that its
  // padding rows and columns (read by the matrix cores against zero entries
  // of K) are zero, not stale values.
  for (int i = lane; i < 3 * KPL * RB; i += 64) S.B[i] = T(0);
  __syncthreads();

  // Cauchy-Kovalevskaya recursion.  Y_e = D^{i-1} A*_e^T on the vector ALUs:
  // lane (e, p) keeps row p of A*_e in registers and walks half of the modes,
  // so that the D rows it reads are broadcast to the lanes sharing a mode.
  constexpr int LH = (L + 1) / 2;
  const int pr = lane % 30, half = lane / 30;
  const int pe = pr / 10, pp = pr % 10;
  T Arow[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) Arow[q] = S.A[pe * 100 + pp * 10 + q];
#pragma unroll
  for (int i = 1; i <= N; ++i) {
    if (half < 2) {
      const int l0 = half * LH, l1 = half ? L : LH;
      for (int l = l0; l < l1; ++l) {
        const T* Dr = &S.D[(i - 1) % ND][l * DS];
        T s = T(0);
#pragma unroll
        for (int q = 0; q < 10; ++q) s += Dr[q] * Arow[q];
        S.B[(pe * KPL + l) * RB + pp] = s;
      }
    }
    __syncthreads();
    Acc C[MT];
    zero_C<P, MT>(C);
    wave_gemm<P, MT, 3 * KSL, RB, 3 * KSL, RB == R ? 16 : 10>(a.Kpk, S.B, C, lane);
    // damage source at t_n, projected on the modes in the same accumulators
    // (column 9; the accurate precision's inputs, FP32 accumulation in the
    // BF16 form): D^1 = -(sum_e K^e Y_e) + P r
    if (i == 1) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        wave_gemm_col9<PA_, MT, KSQA>(a.Ppk + (size_t)c * MT * KSQA * 64, S.R_ + 64 * c, C, lane);
    }
    store_C<P, MT, DS>(C, S.D[i % ND], L, T(-1), lane);
    __syncthreads();
    if constexpr (REGS) {
#pragma unroll
      for (int j = 0; j < DPL; ++j) dreg[i * DPL + j] = S.D[i % ND][lane + 64 * j];
    }
  }
}

// The predictor's results kept by an earlier launch of k_predict on the
// same state (D^1..D^N and the cell-averaged tangent): load them instead of
// recomputing them.  Leaves S (and dreg) as predictor_stage does, except S.R_.
template <int N, int P, int ND, bool REGS, int AW>
__device__ inline void predictor_restore(const StepArgs<P>& a, long long e,
                                         PredLDS<N, P, ND, AW>& S,
                                         const MatP<typename Prec<P>::T>& m,
                                         const typename Prec<P>::T* Dk,
                                         const typename Prec<P>::T* Ak, int lane,
                                         typename Prec<P>::T* dreg) {
  using T = typename Prec<P>::T;
  using SL = PredLDS<N, P, ND, AW>;
  constexpr int L = Dims<N>::L;
  constexpr int KPL = SL::KPL, DS = SL::DS, DPL = SL::DPL;
  static_assert(REGS ? ND == 1 : ND == N + 1, "one buffer with register copies, or all");
  for (int i = lane; i < KPL * DS; i += 64) S.D[0][i] = T(0);
  const T* U9 = a.U9 + e * 9 * L;
  const T* De = Dk + (size_t)e * N * KPL * 16;
  if constexpr (REGS) {
#pragma unroll
    for (int i = 1; i <= N; ++i)
#pragma unroll
      for (int j = 0; j < DPL; ++j) dreg[i * DPL + j] = De[(i - 1) * KPL * 16 + lane + 64 * j];
  } else {
    for (int i = lane; i < N * KPL * 16; i += 64) (&S.D[1][0])[i] = De[i];
  }
  if (lane < 48) S.Acc[lane] = Ak[e * 48 + lane];
  if (lane < 9) S.J[lane] = (T)a.geo[e * 16 + lane];
  __syncthreads();
  for (int i = lane; i < 10 * L; i += 64) {
    const int p = i / L, l = i - p * L;
    S.D[0][l * DS + p] = p < 9 ? U9[i] : (T)a.Ua[e * L + l];
  }
  build_Astar<N, P>(S, m, lane);
  __syncthreads();
  if constexpr (REGS) {
#pragma unroll
    for (int j = 0; j < DPL; ++j) dreg[j] = S.D[0][lane + 64 * j];
  }
}

// LDS derivative buffers of the forward predictor: one plus registers up to
// degree 3 (the smaller LDS footprint lets more wavefronts share a compute
// unit), all of them at degree 4 (the register copy would not fit: 45 values
// per lane).
template <int N, int P> struct FwdRegs {
  static constexpr bool value = N <= 3 || P != PREC_F64;
  static constexpr int ND = value ? 1 : N + 1;
};


// Launch shapes of the two halves of the element update.  The prediction
// keeps the derivatives in registers (45 values per lane at degree 4 in FP32)
// with one LDS buffer; the volume half holds only per-point time integrals.
// Degree 4: 3 wavefronts per SIMD (151 registers).  At 4 the budget of 128
// spills 22 registers per lane: the FP32 prediction ran 93.3 against 95.2 ms
// on the 5.3 M-tet step, but its scratch traffic doubled the kernel's HBM
// bytes (1.0e11 against 4.6e10 algorithmic); the split-BF16 one was slower
// outright (90.6 against 82.2 ms).
template <int N, int P> struct PredWaves {
  static constexpr int value = !FwdRegs<N, P>::value ? 1 : (P == PREC_F64 ? 2 : (N <= 3 ? 5 : 3));
};
// (Split-BF16 volume at degree 4: 3 wavefronts per SIMD, where its 162
// registers fit; at 4 the budget of 128 spills.)
template <int N, int P> struct VolWaves {
  static constexpr int value = P == PREC_F64 ? (N <= 3 ? 4 : 2) : (N <= 3 ? 6 : (P == PREC_BF16 ? 3 : 2));
};

// Prediction (Appendix A.1): Cauchy-Kovalevskaya derivatives of the element
// and the Taylor sums at the Gauss-Legendre time points (Eq. taylor_expansion),
// written to HBM in the [l][16] fragment layout (padding rows and columns
// zero); the derivatives and the cell-averaged tangent also go to Dkeep /
// Akeep when the adjoint's replay asks for them.
template <int N, int P, class LW = CdmLaw>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PredWaves<N, P>::value)))
void k_predict(StepArgs<P> a) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using DM = Dims<N>;
  constexpr int L = DM::L, Nt = DM::Nt;
  constexpr int KS = PR::KS, KPL = round_up(L, KS);
  constexpr bool REGS = FwdRegs<N, P>::value;
  constexpr int ND = FwdRegs<N, P>::ND;
  using SL = PredLDS<N, P, ND, 2>;
  constexpr int DPL = SL::DPL;
  static_assert(SL::DS == 16, "time-point states are copied to HBM row by row");
  __shared__ SL S;
  T dreg[(N + 1) * DPL];

  const int lane = threadIdx.x;
  const long long e = elem_index(a);
  if (e < 0) return;
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  predictor_stage<N, P, ND, REGS, 2, LW>(a, e, S, m, lane, dreg);
  // D^i[idx] for idx = lane + 64 j
  auto Dv = [&](int i, int j) -> T {
    if constexpr (REGS)
      return dreg[i * DPL + j];
    else
      return S.D[i][lane + 64 * j];
  };
  if (a.Dkeep) {
    T* De = a.Dkeep + (size_t)e * N * KPL * 16;
#pragma unroll
    for (int i = 1; i <= N; ++i)
#pragma unroll
      for (int j = 0; j < DPL; ++j) De[(i - 1) * KPL * 16 + lane + 64 * j] = Dv(i, j);
    if (a.Akeep && lane < 48) a.Akeep[e * 48 + lane] = S.Acc[lane];
  }
  T* Uzo = a.Uz + (size_t)e * DM::UZE;
#pragma unroll
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
      const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
      if (l < L && p < 10) Uzo[z * DM::UZT + l * 10 + p] = v;
    }
  }
}

// ---- Picard-iteration predictor --------------------------------------------------
// The alternative to the linearised Cauchy-Kovalevskaya prediction named in the
// paper's Discussion (Section 5.1).  The element-local evolution that the
// recursion differentiates, taken in strong form without linearisation,
//   dU/dt = R(U) = - sum_e KP^e G^e(U) + Pw r(U),
//   G^e = sum_d Theta^-1_ed F^d(V U) at the volume points, KP^e = K^e Pw,
// is solved on the Gauss-Legendre time points by Picard iteration of the
// collocation equations U_z = U^n + dt sum_j Om_zj R(U_j), from U_z = U^n.
template <int P> struct PicardArgs {
  using T = typename Prec<P>::T;
  const typename Prec<P>::AF* KPpk;   // KP^e per 64-point chunk, packed like Spk
  int iters;
  T om[8][8];
};

template <int N, int P> struct PicardLDS {
  using T = typename Prec<P>::T;
  static constexpr int R = Lds<T>::RS;
  static constexpr int KPL = round_up(Dims<N>::L, Prec<P>::KS);
  static constexpr int XS = 64 * R > KPL * 16 ? 64 * R : KPL * 16;
  T X[XS];                            // nodal values / integrands of one chunk, R(U_j)
  T Uz[Dims<N>::Nt][KPL * 16];        // the current iterate U_z, [l][16]
  T R_[64];                           // damage rate at the points of one chunk
  T J[9];                             // Theta^-1
};

template <int N, int P> struct PicardWaves {
  static constexpr int value = P == PREC_F64 ? (N <= 2 ? 3 : 2) : (N <= 2 ? 4 : (N == 3 ? 3 : 2));
};

template <int N, int P, class LW = CdmLaw>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PicardWaves<N, P>::value)))
void k_predict_picard(StepArgs<P> a, PicardArgs<P> pa) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  constexpr int PA_ = Accurate<P>::value;
  using PA = Prec<PA_>;
  using DM = Dims<N>;
  constexpr int L = DM::L, Q = DM::Q, Nt = DM::Nt, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  constexpr int KSQ = 64 / KS, KSQA = 64 / PA::KS;
  constexpr int DPL = KPL * 16 / 64;
  using SL = PicardLDS<N, P>;
  constexpr int R = SL::R;
  __shared__ SL S;
  T* const sX = S.X;

  const int lane = threadIdx.x;
  const long long e = elem_index(a);
  if (e < 0) return;
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  if (lane < 9) S.J[lane] = (T)a.geo[e * 16 + lane];
  const T ir = T(1) / m.rho;
  const T dt = (T)a.dt;

  // U^n in the [l][16] layout, lane + 64 j (padding rows and columns zero)
  T u0[DPL];
  const T* U9 = a.U9 + e * 9 * L;
#pragma unroll
  for (int j = 0; j < DPL; ++j) {
    const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
    u0[j] = (l < L && p < 10) ? (p < 9 ? U9[p * L + l] : (T)a.Ua[e * L + l]) : T(0);
  }
#pragma unroll
  for (int z = 0; z < Nt; ++z)
#pragma unroll
    for (int j = 0; j < DPL; ++j) S.Uz[z][lane + 64 * j] = u0[j];

  T un[Nt][DPL];                      // the next iterate, accumulated
  for (int it = 0; it < pa.iters; ++it) {
#pragma unroll
    for (int z = 0; z < Nt; ++z)
#pragma unroll
      for (int j = 0; j < DPL; ++j) un[z][j] = u0[j];
    for (int jt = 0; jt < Nt; ++jt) {
      __syncthreads();
      Acc Rc[MT];
      zero_C<P, MT>(Rc);
#pragma unroll 1
      for (int c = 0; c < NCH; ++c) {
        // nodal values of U_jt at the chunk's points, pointwise flux as G^e
        // of the reference directions, damage rate
        Acc C[4];
        zero_C<P, 4>(C);
        wave_gemm_tiles<P, 4, KSL, 16>(a.Vpk + (size_t)c * 4 * KSL * 64, S.Uz[jt], C, lane);
        store_C<P, 4>(C, sX, 64, T(1), lane);
        __syncthreads();
        const bool on = 64 * c + lane < Q;
        T u[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
        T sig[6];
        const T r = LW::stress_rate(u, m, law, sig);
        S.R_[lane] = on ? r : T(0);
        // R += -sum_e KP^e G^e over this chunk, direction by direction
#pragma unroll 1
        for (int ee = 0; ee < 3; ++ee) {
          T Jr[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) Jr[d] = S.J[ee * 3 + d];
          T G[9];
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            const int ii = kVI[p], jj = kVJ[p];
            G[p] = T(-0.5) * (Jr[jj] * u[6 + ii] + Jr[ii] * u[6 + jj]);
          }
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) {
            T t = T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) t += Jr[d] * sig[sym_idx(ii, d)];
            G[6 + ii] = -ir * t;
          }
          __syncthreads();
#pragma unroll
          for (int p = 0; p < 16; ++p) sX[lane * R + p] = (on && p < 9) ? -G[p] : T(0);
          __syncthreads();
          wave_gemm_tiles<P, MT, KSQ>(pa.KPpk + (size_t)(ee * NCH + c) * MT * KSQ * 64, sX, Rc,
                                      lane);
        }
        // + Pw r in the damage column
        wave_gemm_col9<PA_, MT, KSQA>(a.Ppk + (size_t)c * MT * KSQA * 64, S.R_, Rc, lane);
        __syncthreads();
      }
      // the next iterate: U_z += dt Om_z,jt R(U_jt) for every z
      store_C<P, MT, 16>(Rc, sX, KPL, T(1), lane);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < DPL; ++j) {
        const int idx = lane + 64 * j;
        const T rv = (idx & 15) < 10 ? sX[idx] : T(0);
#pragma unroll
        for (int z = 0; z < Nt; ++z) un[z][j] += dt * pa.om[z][jt] * rv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < Nt; ++z)
#pragma unroll
      for (int j = 0; j < DPL; ++j) S.Uz[z][lane + 64 * j] = un[z][j];
  }
  __syncthreads();
  T* Uzo = a.Uz + (size_t)e * DM::UZE;
#pragma unroll
  for (int z = 0; z < Nt; ++z)
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
      if (l < L && p < 10) Uzo[z * DM::UZT + l * 10 + p] = S.Uz[z][idx];
    }
}

// LDS of the volume half: nodal values / integrands of one 64-point chunk, the
// damage-rate integrals, Theta^-1, and the partial update before it is stored.
template <int N, int P> struct VolLDS {
  using T = typename Prec<P>::T;
  static constexpr int R = Lds<T>::RS;
  static constexpr int KPL = round_up(Dims<N>::L, Prec<P>::KS);
  static constexpr int XS = 64 * R > KPL * 16 ? 64 * R : KPL * 16;
  T X[XS];
  T W[KPL * 16];          // the time-point state being evaluated, [l][16]
  T R_[Dims<N>::NCH * 64];
};

// Volume and source terms (Appendix A.2, Eqs. 3rd term, rhs term) from the
// time-point states written by k_predict: stress and damage rate at every
// (z, q), accumulated as time integrals of velocity and stress per point (the
// flux is linear in both, so the Jacobian and the stiffness contraction are
// applied once); volume contraction + source projection; partial update
// U^n + volume + source written to W (the faces are subtracted later).
template <int N, int P, class LW = CdmLaw>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(VolWaves<N, P>::value)))
void k_volume(StepArgs<P> a) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  constexpr int PA_ = Accurate<P>::value;
  using PA = Prec<PA_>;
  using DM = Dims<N>;
  constexpr int L = DM::L, Q = DM::Q, Nt = DM::Nt, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  constexpr int KSQ = 64 / KS, KSQA = 64 / PA::KS;
  using SL = VolLDS<N, P>;
  constexpr int R = SL::R;
  __shared__ SL S;
  T* const sX = S.X;
  T* const sR = S.R_;

  const int lane = threadIdx.x;
  const long long e = elem_index(a);
  if (e < 0) return;
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  T Ji[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ji[k] = (T)a.geo[e * 16 + k];
  const T* Uze = a.Uz + (size_t)e * DM::UZE;
  // time-point states go through LDS one at a time, into [l][16] with the
  // padding rows and columns zero (set here, never written again); the next
  // one's loads are in flight while the current one is evaluated
  constexpr int ZPL = (DM::UZT + 63) / 64;
  for (int i = lane; i < KPL * 16; i += 64) S.W[i] = T(0);
  auto uz_at = [&](int z, int j) -> T {
    const int idx = lane + 64 * j;
    return idx < DM::UZT ? Uze[z * DM::UZT + idx] : T(0);
  };
  T nxt[ZPL];
#pragma unroll
  for (int j = 0; j < ZPL; ++j) nxt[j] = uz_at(0, j);

  T vs[NCH][3], ss[NCH][6], sacc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    sacc[c] = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) vs[c][k] = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) ss[c][k] = T(0);
  }
  for (int z = 0; z < Nt; ++z) {
    const T g = a.gamma[z];
#pragma unroll
    for (int j = 0; j < ZPL; ++j) {
      const int idx = lane + 64 * j;
      if (idx < DM::UZT) S.W[(idx / 10) * 16 + idx % 10] = nxt[j];
    }
    if (z + 1 < Nt) {
#pragma unroll
      for (int j = 0; j < ZPL; ++j) nxt[j] = uz_at(z + 1, j);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      Acc C[4];
      zero_C<P, 4>(C);
      wave_gemm_tiles<P, 4, KSL, 16>(a.Vpk + (size_t)c * 4 * KSL * 64, S.W, C, lane);
      store_C<P, 4>(C, sX, 64, T(1), lane);
      __syncthreads();
      const int q = 64 * c + lane;
      if (q < Q) {
        T u[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) u[k] = sX[lane * R + k];
        T sig[6];
        sacc[c] += g * LW::stress_rate(u, m, law, sig);
#pragma unroll
        for (int k = 0; k < 6; ++k) ss[c][k] += g * sig[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) vs[c][k] += g * u[6 + k];
      }
      __syncthreads();
    }
  }

  // volume contraction Vol = sum_e Sw^e G^e and damage source integral, with
  // G^e_(ij) = -(Theta^-1_ej v_i + Theta^-1_ei v_j)/2 and
  // G^e_(v_i) = -(1/rho) sum_d Theta^-1_ed sigma_id of the time integrals
  const T ir = T(1) / m.rho;
  Acc Vc[MT];
  zero_C<P, MT>(Vc);
#pragma unroll
  for (int ee = 0; ee < 3; ++ee) {
    const T* Jr = Ji + ee * 3;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      T G[16];
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int ii = kVI[p], jj = kVJ[p];
        G[p] = T(-0.5) * (Jr[jj] * vs[c][ii] + Jr[ii] * vs[c][jj]);
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        T t = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) t += Jr[d] * ss[c][sym_idx(ii, d)];
        G[6 + ii] = -ir * t;
      }
#pragma unroll
      for (int p = 9; p < 16; ++p) G[p] = T(0);
#pragma unroll
      for (int p = 0; p < 16; ++p) sX[lane * R + p] = G[p];
      __syncthreads();
      wave_gemm_tiles<P, MT, KSQ>(a.Spk + (size_t)(ee * NCH + c) * MT * KSQ * 64, sX, Vc, lane);
      __syncthreads();
    }
  }
  // damage source integral in the same accumulators: column 9 of the volume
  // contraction is zero (no damage flux), the source takes its place
#pragma unroll
  for (int c = 0; c < NCH; ++c) sR[64 * c + lane] = sacc[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCH; ++c)
    wave_gemm_col9<PA_, MT, KSQA>(a.Ppk + (size_t)c * MT * KSQA * 64, sR + 64 * c, Vc, lane);
  store_C<P, MT, 16>(Vc, sX, L, (T)a.dt, lane);
  __syncthreads();
  // U^n + volume for the nine wave quantities; the damage increment joins the
  // FP64 damage plane
  const T* U9 = a.U9 + e * 9 * L;
  T* W9 = a.W9 + e * 9 * L;
  for (int idx = lane; idx < 9 * L; idx += 64) {
    const int p = idx / L, l = idx - p * L;
    W9[idx] = U9[idx] + sX[l * 16 + p];
  }
  if (lane < L) a.Wa[e * L + lane] = a.Ua[e * L + lane] + (double)sX[lane * 16 + 9];
}


// ---- volume and source terms, three elements per wavefront -----------------------
// The same computation as k_volume with the 10 quantities of three elements
// side by side in the columns of every reference-matrix contraction (column
// 10 j + p for element j, quantity p; 30 of 32 columns used): each A fragment
// feeds two matrix-core products for three elements instead of one product
// (10 of 16 columns) for one.
// Column 32 of X (the padding column, never written by the matrix stages)
// holds Theta^-1 of the three elements in rows 0..26 and their materials in
// rows 27..50, so that the LDS of one wavefront stays within a twelfth of a
// compute unit's (three wavefronts per SIMD at degree 4).
template <int N, int P> struct Vol3LDS {
  using T = typename Prec<P>::T;
  static constexpr int RS = 33;                     // 32 columns, odd stride
  static constexpr int KPL = round_up(Dims<N>::L, Prec<P>::KS);
  static constexpr int XR = 64 > KPL ? 64 : KPL;
  static_assert(XR >= 51, "Theta^-1 and materials fit the padding column of X");
  T X[XR * RS];                                     // point values / integrands of a chunk
  T W[KPL * RS];                                    // time-point states of the three elements
  __device__ T& J(int j, int k) { return X[(9 * j + k) * RS + 32]; }
  __device__ T& M(int j, int k) { return X[(27 + 8 * j + k) * RS + 32]; }
};

template <int N, int P, class LW = CdmLaw>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_volume3(StepArgs<P> a) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  constexpr int PA_ = Accurate<P>::value;
  using PA = Prec<PA_>;
  using DM = Dims<N>;
  constexpr int L = DM::L, Q = DM::Q, Nt = DM::Nt, NCH = DM::NCH, MT = DM::MT;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  constexpr int KSQ = 64 / KS, KSQA = 64 / PA::KS;
  constexpr int DPL = KPL * 16 / 64;
  using SL = Vol3LDS<N, P>;
  constexpr int RS = SL::RS;
  __shared__ SL S;
  T* const sX = S.X;
  T* const sW = S.W;

  const int lane = threadIdx.x;
  const long long n = a.elist ? a.nlist : a.E;
  const long long ng = (n + 2) / 3;
  const long long per = (ng + 7) / 8;
  const long long g = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= ng) return;
  long long el[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const long long i = 3 * g + j;
    el[j] = i < n ? (a.elist ? (long long)a.elist[i] : i) : -1;
  }
  const Law<T> law{a.amax, a.smin};
  if (lane < 24) {
    const long long ej = el[lane / 8] >= 0 ? el[lane / 8] : el[0];
    S.M(lane / 8, lane % 8) = (T)a.mat[ej * 8 + lane % 8];
  }
  auto mat_of = [&](int j) {
    MatP<T> mm;
    mm.rho = S.M(j, 0);
    mm.lam = S.M(j, 1);
    mm.mu = S.M(j, 2);
    mm.gr = S.M(j, 3);
    mm.xi0 = S.M(j, 4);
    mm.cd = S.M(j, 5);
    return mm;
  };
  if (lane < 27) {
    const long long ej = el[lane / 9];
    S.J(lane / 9, lane % 9) = ej >= 0 ? (T)a.geo[ej * 16 + lane % 9] : T(0);
  }
  for (int i = lane; i < KPL * RS; i += 64) sW[i] = T(0);


  T vs[NCH][3][3], ss[NCH][3][6], sacc[NCH][3];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      sacc[c][j] = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) vs[c][j][k] = T(0);
#pragma unroll
      for (int k = 0; k < 6; ++k) ss[c][j][k] = T(0);
    }
  for (int z = 0; z < Nt; ++z) {
    const T gz = a.gamma[z];
    __syncthreads();
    // the three elements' time-point states, quantities side by side
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      // (rows L..KPL-1 keep the zeros set at the start)
      const T* Uz = a.Uz + (size_t)(el[j] >= 0 ? el[j] : el[0]) * DM::UZE + z * DM::UZT;
#pragma unroll
      for (int q = 0; q < (DM::UZT + 63) / 64; ++q) {
        const int idx = lane + 64 * q;
        if (idx < DM::UZT) sW[(idx / 10) * RS + 10 * j + idx % 10] = el[j] >= 0 ? Uz[idx] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      Acc C[4][2];
      zero_C2<P, 4>(C);
      wave_gemm2<P, 4, KSL, RS>(a.Vpk + (size_t)c * 4 * KSL * 64, sW, C, lane);
      store_C2<P, 4, RS>(C, sX, 64, T(1), lane);
      __syncthreads();
      if (64 * c + lane < Q) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T u[10];
#pragma unroll
          for (int k = 0; k < 10; ++k) u[k] = sX[lane * RS + 10 * j + k];
          T sig[6];
          sacc[c][j] += gz * LW::stress_rate(u, mat_of(j), law, sig);
#pragma unroll
          for (int k = 0; k < 6; ++k) ss[c][j][k] += gz * sig[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) vs[c][j][k] += gz * u[6 + k];
        }
      }
      __syncthreads();
    }
  }

  // damage source first (its accumulators are free again before those of
  // the volume contraction are taken): the three elements' rate integrals in
  // columns 0..2 of one 16-column tile, projected, times dt, to columns 0..2
  // of W (the damage columns 10 j + 9 of the volume contraction are zero: no
  // damage flux)
  {
    typename PA::Acc Sc[MT];
    zero_C<PA_, MT>(Sc);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) sX[lane * RS + k] = k < 3 ? sacc[c][k] : T(0);
      __syncthreads();
      wave_gemm<PA_, MT, KSQA, RS>(a.Ppk + (size_t)c * MT * KSQA * 64, sX, Sc, lane);
    }
    store_C<PA_, MT, RS, 3>(Sc, sW, L, (T)a.dt, lane);
  }

  // volume contraction sum_e Sw^e G^e
  Acc Vc[MT][2];
  zero_C2<P, MT>(Vc);
#pragma unroll 1
  for (int ee = 0; ee < 3; ++ee) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T ir = T(1) / S.M(j, 0);
        T Jr[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) Jr[d] = S.J(j, ee * 3 + d);
        T* row = sX + lane * RS + 10 * j;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
          const int ii = kVI[p], jj = kVJ[p];
          row[p] = T(-0.5) * (Jr[jj] * vs[c][j][ii] + Jr[ii] * vs[c][j][jj]);
        }
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          T t = T(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) t += Jr[d] * ss[c][j][sym_idx(ii, d)];
          row[6 + ii] = -ir * t;
        }
        row[9] = T(0);
      }
      sX[lane * RS + 30] = T(0);
      sX[lane * RS + 31] = T(0);
      __syncthreads();
      wave_gemm2<P, MT, KSQ, RS>(a.Spk + (size_t)(ee * NCH + c) * MT * KSQ * 64, sX, Vc, lane);
      __syncthreads();
    }
  }
  store_C2<P, MT, RS>(Vc, sX, L, (T)a.dt, lane);
  __syncthreads();
  // U^n + volume for the nine wave quantities; the damage increment joins the
  // FP64 damage plane
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (el[j] < 0) continue;
    const long long e = el[j];
    const T* U9 = a.U9 + e * 9 * L;
    T* W9 = a.W9 + e * 9 * L;
    for (int idx = lane; idx < 9 * L; idx += 64) {
      const int p = idx / L, l = idx - p * L;
      W9[idx] = U9[idx] + sX[l * RS + 10 * j + p];
    }
    if (lane < L) a.Wa[e * L + lane] = a.Ua[e * L + lane] + (double)sW[lane * RS + j];
  }
}

// One wavefront per face (interior faces once, boundary faces once): traces of
// both sides at the shared face points for every time point, LLF (or
// boundary) flux with the normal of the face's first element, time quadrature.
// Writes sum_z gamma_z F*(t_z) at the Ns face points, [face][Ns][10].
// Trace contractions of the face kernel with each trace-matrix fragment shared
// by all time points (FP32 accumulators: 40 registers per side at degree 4).
template <int P> struct FaceSharedA {
  static constexpr bool value = P != PREC_F64;
};

// Degree 4 (c5 step, ms): FP32 faces 56.7 with the odd trace stride 11 at 3
// wavefronts per SIMD against 57.9 with stride 10 at 4 (LDS within a
// sixteenth of the compute unit's); split-BF16 faces 46.8 with stride 10 at 4
// against 50.0.
template <int N, int P> struct FaceWaves {
  static constexpr int value =
      N >= 4 ? (P == PREC_F64 ? 2 : (P == PREC_BF16 ? 4 : 3)) : (P == PREC_F64 ? 4 : 7);
  static constexpr int stride = N >= 4 && P == PREC_BF16 ? 10 : 11;
};

template <int N, int P, class LW = CdmLaw>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FaceWaves<N, P>::value)))
void k_face_flux(StepArgs<P> a, const int* faces, long long nfaces, typename Prec<P>::T* fflux,
                 const int* flist) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  constexpr int L = DM::L, Ns = DM::Ns, Nt = DM::Nt, NST = DM::NST;
  constexpr int KS = PR::KS, KPL = round_up(L, KS), KSL = KPL / KS;
  // traces keep only the 10 quantities: an odd row stride reads one row per
  // lane without bank conflicts and halves the LDS of the 16-column layout
  constexpr int R = FaceWaves<N, P>::stride;
  constexpr int TS = Ns * R;            // rows beyond Ns are never stored
  __shared__ T sTm[Nt * TS];
  __shared__ T sTp[Nt * TS];

  const int lane = threadIdx.x;
  long long fid = elem_of_block(nfaces);
  if (fid >= nfaces) return;
  if (flist) fid = flist[fid];
  const int ef = faces[fid * 2], of = faces[fid * 2 + 1];
  const long long e = ef >> 2;
  const int f = ef & 3;
  const int w = a.conn[ef * 2 + 1];
  const int kind = conn_kind(w), sp = conn_perm(w);
  const Law<T> law{a.amax, a.smin};
  const MatP<T> m = load_mat<T>(a.mat + e * 8);
  const bool inner = kind == 0;
  const long long nb = inner ? (long long)(of >> 2) : e;
  const int nf = inner ? (of & 3) : f, sq = inner ? conn_nperm(w) : sp;
  const T* Uze = a.Uz + (size_t)e * DM::UZE;
  const T* Uzn = a.Uz + (size_t)nb * DM::UZE;
  const typename PR::AF* Fe = a.Fpk + (size_t)(f * 6 + sp) * NST * KSL * 64;
  const typename PR::AF* Fn = a.Fpk + (size_t)(nf * 6 + sq) * NST * KSL * 64;
  if constexpr (FaceSharedA<P>::value) {
    // one side after the other, all time points together: each trace-matrix
    // fragment is loaded once per side instead of once per time point (a
    // boundary face evaluates its own side twice and uses the first)
    Acc C[Nt][NST];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int z = 0; z < Nt; ++z) zero_C<P, NST>(C[z]);
      wave_gemm_shared_a<P, NST, KSL, Nt, 10, DM::UZT>(side ? Fn : Fe, side ? Uzn : Uze, C, lane);
#pragma unroll
      for (int z = 0; z < Nt; ++z)
        store_C<P, NST, R, 10>(C[z], (side ? sTp : sTm) + z * TS, Ns, T(1), lane);
    }
  } else {
    // both sides' traces in one pass, so that the loads of both time-point
    // states are in flight together
#pragma unroll
    for (int z = 0; z < Nt; ++z) {
      Acc C[NST], Cn[NST];
      zero_C<P, NST>(C);
      zero_C<P, NST>(Cn);
      wave_gemm<P, NST, KSL, 10, KSL, 16, false>(Fe, Uze + z * DM::UZT, C, lane);
      wave_gemm<P, NST, KSL, 10, KSL, 16, false>(Fn, Uzn + z * DM::UZT, Cn, lane);
      store_C<P, NST, R, 10>(C, sTm + z * TS, Ns, T(1), lane);
      store_C<P, NST, R, 10>(Cn, sTp + z * TS, Ns, T(1), lane);
    }
  }
  __syncthreads();
  T n[3];
  n[0] = (T)a.fgeo[(e * 4 + f) * 4 + 0];
  n[1] = (T)a.fgeo[(e * 4 + f) * 4 + 1];
  n[2] = (T)a.fgeo[(e * 4 + f) * 4 + 2];
  const MatP<T> mp = load_mat<T>(a.mat + nb * 8);
  for (int idx = lane; idx < Ns * Nt; idx += 64) {
    const int z = idx / Ns, i = idx - z * Ns;
    T* um = sTm + z * TS + i * R;
    T uM[10], F[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) uM[k] = um[k];
    if (kind == 0) {
      T uP[10];
      const T* up = sTp + z * TS + i * R;
#pragma unroll
      for (int k = 0; k < 10; ++k) uP[k] = up[k];
      llf_flux<LW>(uM, uP, n, m, mp, law, F);
    } else {
      boundary_flux<LW>(kind, uM, n, m, law, F);
    }
    const T g = a.gamma[z];
#pragma unroll
    for (int k = 0; k < 10; ++k) um[k] = g * F[k];
  }
  __syncthreads();
  T* out = fflux + (size_t)fid * Ns * 10;
  for (int idx = lane; idx < Ns * 10; idx += 64) {
    const int i = idx / 10, k = idx - i * 10;
    T s = T(0);
#pragma unroll
    for (int z = 0; z < Nt; ++z) s += sTm[z * TS + i * R + k];
    out[idx] = s;
  }
}


// Face term and final update (Appendix A.2, Eq. time-integrated): each element
// lifts the time-integrated flux of its four faces (negated where it is the
// face's second element: the flux is single valued), scaled by dt |S_f|/|J|,
// and subtracts it from the partial update of k_volume.
template <int N, int P>
__global__ __launch_bounds__(64) void k_lift_update(StepArgs<P> a, const int* fmap,
                                                    const typename Prec<P>::T* fflux) {
  using PR = Prec<P>;
  using T = typename PR::T;
  using Acc = typename PR::Acc;
  using DM = Dims<N>;
  constexpr int L = DM::L, Ns = DM::Ns, MT = DM::MT;
  constexpr int KS = PR::KS;
  constexpr int KPN = round_up(Ns, KS), KSN = KPN / KS;
  constexpr int R = Lds<T>::RS;
  constexpr int FS = KPN * R > MT * 16 * R ? KPN * R : MT * 16 * R;
  __shared__ T sF[FS];

  constexpr int FPL = (Ns * 10 + 63) / 64;   // flux values per lane and face
  constexpr int WPL = (9 * L + 63) / 64;     // partial-update values per lane

  const int lane = threadIdx.x;
  const long long e = elem_index(a);
  if (e < 0) return;
  // every HBM load is issued before the first use: the four faces' fluxes
  // (gathered by face) and the partial update.  Under local time stepping a
  // face shared with the finer cluster brings the flux integral that cluster
  // accumulated over its two steps (already scaled by its step), and clears it.
  T fv[4][FPL], sc[4];
  int sp[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int fm = fmap[e * 4 + f];
    sp[f] = conn_perm(a.conn[(e * 4 + f) * 2 + 1]);
    const int nb = a.conn[(e * 4 + f) * 2];
    const bool fine = a.lts_c > 0 && nb >= 0 && a.ecl[nb] == a.lts_c - 1;
    sc[f] = (T)((fm & 1 ? -1.0 : 1.0) * a.fgeo[(e * 4 + f) * 4 + 3] * (fine ? 1.0 : a.dt));
    T* fl = (fine ? a.facc : (T*)fflux) + (size_t)(fm >> 1) * Ns * 10;
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
      const int idx = lane + 64 * j;
      fv[f][j] = idx < Ns * 10 ? fl[idx] : T(0);
    }
    if (fine) {
#pragma unroll
      for (int j = 0; j < FPL; ++j) {
        const int idx = lane + 64 * j;
        if (idx < Ns * 10) fl[idx] = T(0);
      }
    }
  }
  T* W9 = a.W9 + e * 9 * L;
  T wv[WPL];
#pragma unroll
  for (int j = 0; j < WPL; ++j) {
    const int idx = lane + 64 * j;
    wv[j] = idx < 9 * L ? W9[idx] : T(0);
  }
  const double wa = lane < L ? a.Wa[e * L + lane] : 0.0;
  for (int i = lane; i < FS; i += 64) sF[i] = T(0);
  Acc Fc[MT];
  zero_C<P, MT>(Fc);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FPL; ++j) {
      const int idx = lane + 64 * j;
      if (idx < Ns * 10) {
        const int i = idx / 10, k = idx - i * 10;
        sF[i * R + k] = sc[f] * fv[f][j];
      }
    }
    __syncthreads();
    wave_gemm<P, MT, KSN>(a.Lpk + (size_t)(f * 6 + sp[f]) * MT * KSN * 64, sF, Fc, lane);
  }
  __syncthreads();
  store_C<P, MT>(Fc, sF, L, T(1), lane);
  __syncthreads();
  bool bad = false;
  T* O9 = (a.O9 ? a.O9 : a.W9) + e * 9 * L;
  double* Oa = a.Oa ? a.Oa : a.Wa;
#pragma unroll
  for (int j = 0; j < WPL; ++j) {
    const int idx = lane + 64 * j;
    if (idx < 9 * L) {
      const int p = idx / L, l = idx - p * L;
      const T v = wv[j] - sF[l * R + p];
      bad |= !isfinite(v);
      O9[idx] = v;
    }
  }
  if (lane < L) {
    const double v = wa - (double)sF[lane * R + 9];
    bad |= !isfinite(v);
    Oa[e * L + lane] = v;
  }
  if (bad) a.flag[0] = 1;
}

// Local time stepping: the state of each listed element at the time points
// t_pred + off + tau_z dt of the cluster being corrected, from its kept
// prediction (D^0 = its state, D^1..D^N kept by k_predict), written to Uz in
// the [l][16] layout; off is the time since the element's own prediction.
// The Taylor sum is formed exactly as in k_predict.
struct ClusterOffsets { double v[8]; };   // time since each cluster's prediction

template <int N, int P>
__global__ __launch_bounds__(64) void k_taylor(StepArgs<P> a, ClusterOffsets offs) {
  using T = typename Prec<P>::T;
  using DM = Dims<N>;
  constexpr int L = DM::L, Nt = DM::Nt;
  constexpr int KPL = round_up(L, Prec<P>::KS), DPL = KPL * 16 / 64;
  const int lane = threadIdx.x;
  const long long e = elem_index(a);
  if (e < 0) return;
  const double off = offs.v[a.ecl[e]];
  const T* U9 = a.U9 + e * 9 * L;
  const T* De = a.Dkeep + (size_t)e * N * KPL * 16;
  T d[N + 1][DPL];
#pragma unroll
  for (int j = 0; j < DPL; ++j) {
    const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
    d[0][j] = (l < L && p < 10) ? (p < 9 ? U9[p * L + l] : (T)a.Ua[e * L + l]) : T(0);
  }
#pragma unroll
  for (int i = 1; i <= N; ++i)
#pragma unroll
    for (int j = 0; j < DPL; ++j) d[i][j] = De[(i - 1) * KPL * 16 + lane + 64 * j];
  T* Uzo = a.Uz + (size_t)e * DM::UZE;
#pragma unroll
  for (int z = 0; z < Nt; ++z) {
    T cz[N + 1];
    cz[0] = T(1);
    const T h = a.tau[z] * (T)a.dt + (T)off;   // as k_predict's when off = 0
#pragma unroll
    for (int i = 1; i <= N; ++i) cz[i] = cz[i - 1] * h / T(i);
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      T v = T(0);
#pragma unroll
      for (int i = 0; i <= N; ++i) v += cz[i] * d[i][j];
      const int idx = lane + 64 * j, l = idx >> 4, p = idx & 15;
      if (l < L && p < 10) Uzo[z * DM::UZT + l * 10 + p] = v;
    }
  }
}

// Local time stepping: faces between the cluster being corrected and the next
// coarser one keep the time integral of their flux for the coarser side:
// acc += dt * flux over the listed faces.
template <class T>
__global__ void k_face_accumulate(long long nlist, const int* flist, int Ns, double dt,
                                  const T* fflux, T* facc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlist * Ns * 10) return;
  const long long f = flist[i / (Ns * 10)];
  const long long k = f * Ns * 10 + i % (Ns * 10);
  facc[k] = (T)((double)facc[k] + dt * (double)fflux[k]);
}

// ---- point sources, receivers, projection, diagnostics ------------------------

__device__ inline double stf_G(int kind, double tau, double p) {
  if (kind == 0) {
    const double aa = (M_PI * p) * (M_PI * p);
    return -exp(-aa * tau * tau) / (2.0 * aa);
  }
  return 0.5 * (tau * (1.0 + erf(tau / p)) + p * exp(-tau * tau / (p * p)) / sqrt(M_PI));
}

struct SrcArgs {
  int nsrc, L;
  const long long* elem;   // [nsrc]
  const double* M6;        // [nsrc][6]
  const double* dphi;      // [nsrc][3][L]  dphi_l/dx_d at the source
  const double* onset;     // [nsrc]
  const double* param;     // [nsrc]
  const double* rhoJ;      // [nsrc]  rho |J| of the host element
  int kind;
  double t0, t1;
  const signed char* ecl;  // cluster of every element, with only_cluster >= 0
  int only_cluster;        // -1: every source; else those in elements of this cluster
};

template <class T>
__global__ void k_sources(SrcArgs s, T* U9) {
  const int idx = threadIdx.x;   // (i, l)
  if (idx >= 3 * s.L) return;
  const int i = idx / s.L, l = idx % s.L;
  for (int k = 0; k < s.nsrc; ++k) {
    if (s.only_cluster >= 0 && s.ecl[s.elem[k]] != s.only_cluster) continue;
    const double dG = stf_G(s.kind, s.t1 - s.onset[k], s.param[k]) -
                      stf_G(s.kind, s.t0 - s.onset[k], s.param[k]);
    const double fac = dG / s.rhoJ[k];
    double v = 0.0;
    for (int j = 0; j < 3; ++j) v += s.M6[k * 6 + sym_idx(i, j)] * s.dphi[(k * 3 + j) * s.L + l];
    T* dst = U9 + (s.elem[k] * 9 + 6 + i) * s.L + l;
    *dst = (T)((double)*dst + fac * v);
  }
}

template <class T>
__global__ void k_receivers(int nrec, int L, const long long* elem, const double* phi,
                            const T* U9, double* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrec * 3) return;
  const int r = idx / 3, c = idx % 3;
  const T* u = U9 + (elem[r] * 9 + 6 + c) * L;
  double s = 0.0;
  for (int l = 0; l < L; ++l) s += phi[r * L + l] * (double)u[l];
  out[idx] = s;
}

// L2 projection of point values [E][Q][10] onto the modes (FP64)
template <class T>
__global__ void k_project(long long E, int L, int Q, const double* Pw, const double* vals, T* U9,
                          double* Ua) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * 10 * L) return;
  const long long e = idx / (10 * L);
  const int p = (int)((idx / L) % 10), l = (int)(idx % L);
  double s = 0.0;
  for (int q = 0; q < Q; ++q) s += Pw[l * Q + q] * vals[(e * Q + q) * 10 + p];
  if (p < 9)
    U9[(e * 9 + p) * L + l] = (T)s;
  else
    Ua[e * L + l] = s;
}

// point values u(x_q) = sum_l phi_l(xi_q) U_l of elements [0, E) at the volume
// quadrature points, FP64, out [E][Q][10]
template <class T>
__global__ void k_point_values(long long E, int L, int Q, const double* V, const T* U9,
                               const double* Ua, double* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * Q * 10) return;
  const long long e = idx / (Q * 10);
  const int q = (int)((idx / 10) % Q), p = (int)(idx % 10);
  double s = 0.0;
  for (int l = 0; l < L; ++l)
    s += V[q * L + l] * (p < 9 ? (double)U9[(e * 9 + p) * L + l] : Ua[e * L + l]);
  out[idx] = s;
}

template <class T>
__global__ void k_to_f64(long long E, int L, const T* U9, const double* Ua, double* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * 10 * L) return;
  const long long e = idx / (10 * L);
  const int p = (int)((idx / L) % 10), l = (int)(idx % L);
  out[idx] = p < 9 ? (double)U9[(e * 9 + p) * L + l] : Ua[e * L + l];
}

template <class T>
__global__ void k_from_f64(long long E, int L, const double* in, T* U9, double* Ua) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * 10 * L) return;
  const long long e = idx / (10 * L);
  const int p = (int)((idx / L) % 10), l = (int)(idx % L);
  if (p < 9)
    U9[(e * 9 + p) * L + l] = (T)in[idx];
  else
    Ua[e * L + l] = in[idx];
}

// energy: one wave per element, lanes over volume points (FP64)
template <class T>
__global__ __launch_bounds__(64) void k_energy(long long E, int L, int Q, const double* V,
                                               const double* wq, const T* U9, const double* Ua,
                                               const double* geo, const double* mat, double amax,
                                               double smin, double* part) {
  const long long e = blockIdx.x;
  const int lane = threadIdx.x;
  if (e >= E) return;
  const MatP<double> m = load_mat<double>(mat + e * 8);
  const Law<double> law{amax, smin};
  double acc = 0.0;
  for (int q = lane; q < Q; q += 64) {
    double u[10];
    for (int p = 0; p < 10; ++p) {
      double s = 0.0;
      for (int l = 0; l < L; ++l)
        s += V[q * L + l] * (p < 9 ? (double)U9[(e * 9 + p) * L + l] : Ua[e * L + l]);
      u[p] = s;
    }
    const double kin = 0.5 * m.rho * (u[6] * u[6] + u[7] * u[7] + u[8] * u[8]);
    acc += wq[q] * (kin + cdm_energy(u, m, law));
  }
  acc = wave_sum(acc);
  if (lane == 0) part[e] = acc * geo[e * 16 + 9];
}

__global__ void k_reduce_sum(long long n, const double* in, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) s += in[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void k_wavespeed(long long E, int L, const double* Ua, const double* mat, double amax,
                            double phi0_mean, int law, double* out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double ab = phi0_mean * Ua[e * L];
  ab = ab < 0.0 ? 0.0 : (ab > amax ? amax : ab);
  if (law == 1) {   // shear modulus (1 - alpha) mu0 (Eq. effective-ivm)
    out[e] = sqrt(1.0 - ab) - 1.0;
    return;
  }
  const double mu = mat[e * 8 + 2];
  double md = mu + ab * mat[e * 8 + 4] * mat[e * 8 + 3];
  md = md > 0.0 ? md : 0.0;
  out[e] = sqrt(md / mu) - 1.0;
}

}  // namespace dgd
