// C-ABI of the MI355X ADER-DG library (see include/dgd.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgd.h"
#include "adjoint_kernels.hpp"
#include "kernels.hpp"
#include "refgen.hpp"

using namespace dgd;

// Partial energy sums of dgd_energy_noalloc (one per element), for callers
// that cannot allocate device memory.  Every GPU the library runs on holds its
// own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr long long kNoallocMaxElems = 1LL << 20;
static __device__ __align__(256) double scratch[kNoallocMaxElems];

namespace {

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;   // device -> address of its scratch

// device address of `scratch` on the current device (looked up once per device)
hipError_t scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = (double*)p;
  *out = (double*)p;
  return hipSuccess;
}

struct Bf16x8 { uint16_t v[8]; };   // high parts of four values, then their low parts

template <int P> struct HostAF;
template <> struct HostAF<PREC_F64> { using type = double; };
template <> struct HostAF<PREC_F32> { using type = float; };
template <> struct HostAF<PREC_BF16> { using type = Bf16x8; };

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

struct dgd_handle {
  int N = 0, prec = 0, device = 0;
  hipStream_t stream = nullptr;
  double* noalloc_part = nullptr;   // this device's static partial-sum buffer
  std::string err;
  RefData ref;
  size_t tsize = 8;  // bytes of the working type
  // reference data on the device
  DevBuf Vpk, Kpk, Spk, Fpk, Lpk, Ppk, Vd, wqd, Pwd, betad, KPpk;
  bool vol3 = false;      // volume terms three elements per wavefront
  int predictor = 0;      // 0: linearised Cauchy-Kovalevskaya, 1: Picard iteration
  int picard_iters = 0;
  // host copies of the connectivity (neighbour of every element face, face list)
  std::vector<int> nbr_h, faces_h;
  std::vector<double> fgeo_h;
  // local time stepping: clusters, base step, per-cluster launch lists
  int nclusters = 0;
  double lts_dt0 = 0.0;
  std::vector<signed char> cl_h;
  DevBuf ecl, Dall, facc;
  std::vector<DevBuf> lts_el, lts_tay, lts_fl, lts_acc;
  std::vector<long long> n_el, n_tay, n_fl, n_acc;
  double lts_tp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int kpl = 0;  // padded mode count of the time-point state layout
  double inv_wsum = 6.0, phi0_mean = 0.0;
  // mesh and material
  long long ne = 0;
  bool have_mesh = false, have_mat = false, have_params = false, have_state = false;
  std::vector<double> X0, Jm, Jinv, detJ;  // host copies for point location
  DevBuf geo, fgeo, conn, mat;
  DevBuf faces, fmap, fflux;   // face list (first side, second side), element -> face, face fluxes
  long long nfaces = 0;
  std::vector<double> rho_h;
  int law = 0;   // 0: continuum damage (Eq. cdb-model), 1: internal variable (Eq. ivm-model)
  // state
  DevBuf U9[2], Ua[2], Uz, flag, tmp;   // tmp: per-call host transfers
  int cur = 0;
  double dt = 0.0, amax = 0.5, t = 0.0;
  long long steps_since_check = 0, check_every = 64;
  // sources and receivers
  int nsrc = 0, srckind = 0;
  DevBuf s_elem, s_M6, s_dphi, s_onset, s_param, s_rhoJ;
  int nrec = 0;
  DevBuf r_elem, r_phi, seis;
  long long nrec_steps = 0, seis_cap = 0;
  // profiling: event pairs per kernel class
  // discrete adjoint: transposed reference data, adjoint state, checkpoints
  DevBuf VTpk, STpk, PTpk, KTpk;
  // FP32 forward operators of a split-BF16 handle, for its FP32 adjoint
  DevBuf Vpk32, Kpk32, Spk32, Fpk32, Lpk32, Ppk32, KPpk32;
  DevBuf lam[2], gtr, gmuf, lzf, gmu, gcd, adjW9, adjWa, dlds, seg9, sega, seguz, segd, segacc, save9, savea;
  DevBuf st9, sta;               // the state U^n handed to dgd_adjoint_step, working precision
  void* uz_override = nullptr;   // time-point states of the step being replayed
  void* d_keep = nullptr;        // where that replay keeps D^1..D^N (or null)
  void* acc_keep = nullptr;      // where it keeps the cell-averaged tangents (or null)
  std::vector<DevBuf> ck9, cka;
  std::vector<double> ck_t;
  long long tape_steps = 0, tape_every = 0, tape_seis0 = 0;
  bool tape = false;
  long long tape_id = 0, tapes_made = 0;   // id of the kept tape (0: none)
  std::vector<double> mat_h;               // host copy of the material table [E][8]
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;

  ~dgd_handle() {
    DevBuf* all[] = {&Vpk, &Kpk, &Spk, &Fpk, &Lpk, &Ppk, &Vd, &wqd, &Pwd, &betad, &geo, &fgeo,
                     &conn, &mat, &faces, &fmap, &fflux, &U9[0], &U9[1], &Ua[0], &Ua[1], &Uz, &flag, &tmp,
                     &s_elem, &s_M6, &s_dphi, &s_onset, &s_param, &s_rhoJ, &r_elem, &r_phi, &seis,
                     &VTpk, &STpk, &PTpk, &KTpk, &lam[0], &lam[1], &gtr, &gmuf, &lzf, &gmu, &gcd, &adjW9,
                     &adjWa, &dlds, &seg9, &sega, &seguz, &segd, &segacc, &save9, &savea, &st9, &sta,
                     &KPpk, &ecl, &Dall, &facc, &Vpk32, &Kpk32, &Spk32, &Fpk32, &Lpk32, &Ppk32,
                     &KPpk32};
    for (DevBuf* b : all) b->release();
    for (DevBuf& b : ck9) b.release();
    for (DevBuf& b : cka) b.release();
    for (auto* v : {&lts_el, &lts_tay, &lts_fl, &lts_acc})
      for (DevBuf& b : *v) b.release();
    for (auto& u : ev_used) {
      (void)hipEventDestroy(u.second.first);
      (void)hipEventDestroy(u.second.second);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

dgd_status fail(dgd_handle* h, dgd_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

dgd_status hip_check(dgd_handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return DGD_OK;
  return fail(h, e == hipErrorOutOfMemory ? DGD_ENOMEM : DGD_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                       \
  do {                                                        \
    dgd_status _s = hip_check((h), (call), #call);            \
    if (_s != DGD_OK) return _s;                              \
  } while (0)

dgd_status dalloc(dgd_handle* h, DevBuf& b, size_t bytes) {
  if (b.n == bytes && b.p) return DGD_OK;
  b.release();
  if (bytes == 0) return DGD_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hip_check(h, e, "hipMalloc");
  }
  b.n = bytes;
  return DGD_OK;
}

template <class V>
dgd_status upload(dgd_handle* h, DevBuf& b, const std::vector<V>& v) {
  dgd_status s = dalloc(h, b, v.size() * sizeof(V));
  if (s != DGD_OK) return s;
  if (v.empty()) return DGD_OK;
  HIPCHK(h, hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DGD_OK;
}

uint16_t bf16_bits(double x) { return f32_to_bf16((float)x); }

float bf16_value(uint16_t b) {
  union { uint32_t u; float f; } v;
  v.u = (uint32_t)b << 16;
  return v.f;
}

// pack A (rows x cols via accessor) into fragment order [tile][kstep][lane]
template <int P, class F>
std::vector<typename HostAF<P>::type> pack_A(F A, int tiles, int ksteps) {
  using AF = typename HostAF<P>::type;
  std::vector<AF> out((size_t)tiles * ksteps * 64);
  constexpr int KS = Prec<P>::KS;
  for (int t = 0; t < tiles; ++t)
    for (int s = 0; s < ksteps; ++s)
      for (int lane = 0; lane < 64; ++lane) {
        const int m = 16 * t + (lane & 15);
        AF& o = out[((size_t)t * ksteps + s) * 64 + lane];
        if constexpr (P == PREC_BF16) {
          // split of the FP32 value into high and low BF16 parts
          for (int j = 0; j < 4; ++j) {
            const float x = (float)A(m, KS * s + 4 * (lane >> 4) + j);
            o.v[j] = bf16_bits(x);
            o.v[4 + j] = bf16_bits(x - bf16_value(o.v[j]));
          }
        } else {
          o = (AF)A(m, KS * s + (lane >> 4));
        }
      }
  return out;
}

template <class V>
void append(std::vector<V>& a, const std::vector<V>& b) {
  a.insert(a.end(), b.begin(), b.end());
}

template <int N, int P>
dgd_status build_packed(dgd_handle* h) {
  using DM = Dims<N>;
  using AF = typename HostAF<P>::type;
  using T = typename Prec<P>::T;
  const RefData& r = h->ref;
  constexpr int KS = Prec<P>::KS, L = DM::L, Q = DM::Q, Ns = DM::Ns;
  constexpr int KPL = round_up(L, KS), KSL = KPL / KS, KPN = round_up(Ns, KS), KSN = KPN / KS;
  std::vector<AF> v, k, s, f, lf, kp;
  for (int c = 0; c < DM::NCH; ++c)
    append(v, pack_A<P>(
                  [&](int m, int kk) {
                    int q = 64 * c + m;
                    return (q < Q && kk < L) ? r.V[(size_t)q * L + kk] : 0.0;
                  },
                  4, KSL));
  k = pack_A<P>(
      [&](int m, int kk) {
        int e = kk / KPL, l = kk % KPL;
        return (m < L && l < L) ? r.K[((size_t)e * L + m) * L + l] : 0.0;
      },
      DM::MT, 3 * KSL);
  for (int e = 0; e < 3; ++e)
    for (int c = 0; c < DM::NCH; ++c) {
      append(s, pack_A<P>(
                    [&](int m, int kk) {
                      int q = 64 * c + kk;
                      return (m < L && q < Q) ? r.Sw[((size_t)e * L + m) * Q + q] : 0.0;
                    },
                    DM::MT, 64 / KS));
      append(kp, pack_A<P>(
                     [&](int m, int kk) {
                       int q = 64 * c + kk;
                       return (m < L && q < Q) ? r.KP[((size_t)e * L + m) * Q + q] : 0.0;
                     },
                     DM::MT, 64 / KS));
    }
  for (int ff = 0; ff < 4; ++ff)
    for (int sp = 0; sp < 6; ++sp) {
      const double* F = &r.F[((size_t)ff * 6 + sp) * Ns * L];
      append(f, pack_A<P>([&](int m, int kk) { return (m < Ns && kk < L) ? F[m * L + kk] : 0.0; },
                          DM::NST, KSL));
      append(lf, pack_A<P>(
                     [&](int m, int kk) {
                       return (m < L && kk < Ns) ? r.beta[kk] * F[kk * L + m] : 0.0;
                     },
                     DM::MT, KSN));
    }
  // damage-source projection in the accurate precision
  constexpr int PA = Accurate<P>::value;
  constexpr int KSQA = 64 / Prec<PA>::KS;
  std::vector<typename HostAF<PA>::type> pp;
  for (int c = 0; c < DM::NCH; ++c)
    append(pp, pack_A<PA>(
                   [&](int m, int kk) {
                     int q = 64 * c + kk;
                     return (m < L && q < Q) ? r.Pw[(size_t)m * Q + q] : 0.0;
                   },
                   DM::MT, KSQA));
  dgd_status st;
  if ((st = upload(h, h->Vpk, v)) || (st = upload(h, h->Kpk, k)) || (st = upload(h, h->Spk, s)) ||
      (st = upload(h, h->Fpk, f)) || (st = upload(h, h->Lpk, lf)) || (st = upload(h, h->Ppk, pp)) ||
      (st = upload(h, h->KPpk, kp)))
    return st;
  if constexpr (P != PREC_BF16) {
    // transposed operators of the discrete adjoint
    std::vector<AF> vt, stt, pt, kt;
    for (int c = 0; c < DM::NCH; ++c) {
      append(vt, pack_A<P>(
                     [&](int m, int kk) {
                       int q = 64 * c + kk;
                       return (m < L && q < Q) ? r.V[(size_t)q * L + m] : 0.0;
                     },
                     DM::MT, 64 / KS));
      append(pt, pack_A<P>(
                     [&](int m, int kk) {
                       int q = 64 * c + m;
                       return (q < Q && kk < L) ? r.Pw[(size_t)kk * Q + q] : 0.0;
                     },
                     4, KSL));
    }
    for (int e = 0; e < 3; ++e) {
      for (int c = 0; c < DM::NCH; ++c)
        append(stt, pack_A<P>(
                        [&](int m, int kk) {
                          int q = 64 * c + m;
                          return (q < Q && kk < L) ? r.Sw[((size_t)e * L + kk) * Q + q] : 0.0;
                        },
                        4, KSL));
      append(kt, pack_A<P>(
                     [&](int m, int kk) {
                       return (m < L && kk < L) ? r.K[((size_t)e * L + kk) * L + m] : 0.0;
                     },
                     DM::MT, KSL));
    }
    if ((st = upload(h, h->VTpk, vt)) || (st = upload(h, h->STpk, stt)) ||
        (st = upload(h, h->PTpk, pt)) || (st = upload(h, h->KTpk, kt)))
      return st;
  }
  h->kpl = KPL;
  (void)sizeof(T);
  return DGD_OK;
}

hipEvent_t take_event(dgd_handle* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// record an event pair around the launch of kernel class k when profiling
template <class F>
void timed(dgd_handle* h, int k, F launch) {
  if (!h->profiling) {
    launch();
    return;
  }
  hipEvent_t a = take_event(h), b = take_event(h);
  if (!a || !b) {
    launch();
    return;
  }
  (void)hipEventRecord(a, h->stream);
  launch();
  (void)hipEventRecord(b, h->stream);
  h->ev_used.push_back({k, {a, b}});
}

template <int N, int P>
StepArgs<P> make_args(dgd_handle* h) {
  using T = typename Prec<P>::T;
  using AF = typename Prec<P>::AF;
  StepArgs<P> a;
  a.E = h->ne;
  const int c = h->cur, n = 1 - h->cur;
  a.U9 = (const T*)h->U9[c].p;
  a.Ua = (const double*)h->Ua[c].p;
  a.W9 = (T*)h->U9[n].p;
  a.Wa = (double*)h->Ua[n].p;
  a.Uz = (T*)(h->uz_override ? h->uz_override : h->Uz.p);
  a.geo = (const double*)h->geo.p;
  a.fgeo = (const double*)h->fgeo.p;
  a.mat = (const double*)h->mat.p;
  a.conn = (const int*)h->conn.p;
  a.Vpk = (const AF*)h->Vpk.p;
  a.Kpk = (const AF*)h->Kpk.p;
  a.Spk = (const AF*)h->Spk.p;
  a.Fpk = (const AF*)h->Fpk.p;
  a.Lpk = (const AF*)h->Lpk.p;
  a.Ppk = (const typename Prec<Accurate<P>::value>::AF*)h->Ppk.p;
  a.wq = (const double*)h->wqd.p;
  a.Dkeep = (T*)h->d_keep;
  a.Akeep = (T*)h->acc_keep;
  a.dt = h->dt;
  a.amax = (T)h->amax;
  a.smin = (T)1e-15;   // guard sqrt(I2) <= 1e-15, i.e. I2 <= 1e-30, in every precision
  a.inv_wsum = (T)h->inv_wsum;
  for (int z = 0; z < 8; ++z) {
    a.tau[z] = z < (int)h->ref.tau.size() ? (T)h->ref.tau[z] : T(0);
    a.gamma[z] = z < (int)h->ref.gamma.size() ? (T)h->ref.gamma[z] : T(0);
  }
  a.flag = (int*)h->flag.p;
  a.elist = nullptr;
  a.nlist = 0;
  a.ecl = nullptr;
  a.lts_c = -1;
  a.facc = nullptr;
  a.O9 = nullptr;
  a.Oa = nullptr;
  return a;
}

// volume and source terms of the listed elements (all without a list): three
// elements per wavefront where that layout is used, else one
template <int N, int P>
void launch_volume(dgd_handle* h, const StepArgs<P>& a, bool ivm) {
  const long long n = a.elist ? a.nlist : a.E;
  if (h->vol3) {
    const long long ng = (n + 2) / 3;
    const dim3 grid((unsigned)(8 * ((ng + 7) / 8)));
    if (ivm)
      hipLaunchKernelGGL((k_volume3<N, P, IvmLaw>), grid, dim3(64), 0, h->stream, a);
    else
      hipLaunchKernelGGL((k_volume3<N, P, CdmLaw>), grid, dim3(64), 0, h->stream, a);
  } else {
    const dim3 grid((unsigned)(8 * ((n + 7) / 8)));
    if (ivm)
      hipLaunchKernelGGL((k_volume<N, P, IvmLaw>), grid, dim3(64), 0, h->stream, a);
    else
      hipLaunchKernelGGL((k_volume<N, P, CdmLaw>), grid, dim3(64), 0, h->stream, a);
  }
}

template <int N, int P>
dgd_status step_impl(dgd_handle* h, long long nsteps) {
  using T = typename Prec<P>::T;
  const long long per = (h->ne + 7) / 8;
  const dim3 grid((unsigned)(8 * per)), block(64);
  const bool ivm = h->law == 1;
  for (long long it = 0; it < nsteps; ++it) {
    StepArgs<P> a = make_args<N, P>(h);
    timed(h, 0, [&] {
      if (h->predictor == 1) {
        PicardArgs<P> pa;
        pa.KPpk = (const typename Prec<P>::AF*)h->KPpk.p;
        pa.iters = h->picard_iters > 0 ? h->picard_iters : N + 1;
        for (int z = 0; z < 8; ++z)
          for (int j = 0; j < 8; ++j)
            pa.om[z][j] = (z < h->ref.Nt && j < h->ref.Nt) ? (T)h->ref.Om[z * h->ref.Nt + j] : T(0);
        if (ivm)
          hipLaunchKernelGGL((k_predict_picard<N, P, IvmLaw>), grid, block, 0, h->stream, a, pa);
        else
          hipLaunchKernelGGL((k_predict_picard<N, P, CdmLaw>), grid, block, 0, h->stream, a, pa);
      } else if (ivm) {
        hipLaunchKernelGGL((k_predict<N, P, IvmLaw>), grid, block, 0, h->stream, a);
      } else {
        hipLaunchKernelGGL((k_predict<N, P, CdmLaw>), grid, block, 0, h->stream, a);
      }
    });
    timed(h, 9, [&] { launch_volume<N, P>(h, a, ivm); });
    const long long fper = (h->nfaces + 7) / 8;
    timed(h, 1, [&] {
      if (ivm)
        hipLaunchKernelGGL((k_face_flux<N, P, IvmLaw>), dim3((unsigned)(8 * fper)), block, 0,
                           h->stream, a, (const int*)h->faces.p, h->nfaces, (T*)h->fflux.p,
                           (const int*)nullptr);
      else
        hipLaunchKernelGGL((k_face_flux<N, P>), dim3((unsigned)(8 * fper)), block, 0,
                           h->stream, a, (const int*)h->faces.p, h->nfaces, (T*)h->fflux.p,
                           (const int*)nullptr);
    });
    timed(h, 8, [&] {
      hipLaunchKernelGGL((k_lift_update<N, P>), grid, block, 0, h->stream, a,
                         (const int*)h->fmap.p, (const T*)h->fflux.p);
    });
    if (h->nsrc > 0) {
      SrcArgs s;
      s.nsrc = h->nsrc;
      s.L = h->ref.L;
      s.elem = (const long long*)h->s_elem.p;
      s.M6 = (const double*)h->s_M6.p;
      s.dphi = (const double*)h->s_dphi.p;
      s.onset = (const double*)h->s_onset.p;
      s.param = (const double*)h->s_param.p;
      s.rhoJ = (const double*)h->s_rhoJ.p;
      s.kind = h->srckind;
      s.t0 = h->t;
      s.t1 = h->t + h->dt;
      s.ecl = nullptr;
      s.only_cluster = -1;
      timed(h, 2, [&] {
        hipLaunchKernelGGL((k_sources<T>), dim3(1), dim3(3 * h->ref.L), 0, h->stream, s,
                           (T*)h->U9[1 - h->cur].p);
      });
    }
    if (h->nrec > 0) {
      double* out = (double*)h->seis.p + (size_t)h->nrec_steps * h->nrec * 3;
      const int nth = h->nrec * 3;
      timed(h, 3, [&] {
        hipLaunchKernelGGL((k_receivers<T>), dim3((nth + 63) / 64), dim3(64), 0, h->stream,
                           h->nrec, h->ref.L, (const long long*)h->r_elem.p,
                           (const double*)h->r_phi.p, (const T*)h->U9[1 - h->cur].p, out);
      });
      h->nrec_steps += 1;
    }
    HIPCHK(h, hipGetLastError());
    h->cur = 1 - h->cur;
    h->t += h->dt;
  }
  return DGD_OK;
}

// ---------------------------------------------------------------- local time stepping
// One step of cluster c over [t, t + dt0 2^c] (rate-2 clusters, the finer
// cluster's two steps nested inside; see dgd_set_clusters).
template <int N, int P>
dgd_status lts_advance(dgd_handle* h, int c, double t) {
  using T = typename Prec<P>::T;
  const dim3 block(64);
  auto grid_of = [](long long n) { return dim3((unsigned)(8 * ((n + 7) / 8))); };
  const double dtc = h->lts_dt0 * (double)(1LL << c);
  StepArgs<P> a = make_args<N, P>(h);
  a.ecl = (const signed char*)h->ecl.p;
  a.Dkeep = (T*)h->Dall.p;
  a.Akeep = nullptr;
  a.dt = dtc;
  const bool ivm = h->law == 1;
  if (h->n_el[c] > 0) {
    a.elist = (const int*)h->lts_el[c].p;
    a.nlist = h->n_el[c];
    timed(h, 0, [&] {
      if (ivm)
        hipLaunchKernelGGL((k_predict<N, P, IvmLaw>), grid_of(a.nlist), block, 0, h->stream, a);
      else
        hipLaunchKernelGGL((k_predict<N, P, CdmLaw>), grid_of(a.nlist), block, 0, h->stream, a);
    });
    HIPCHK(h, hipGetLastError());
  }
  h->lts_tp[c] = t;
  dgd_status s;
  if (c > 0) {
    if ((s = lts_advance<N, P>(h, c - 1, t)) || (s = lts_advance<N, P>(h, c - 1, t + 0.5 * dtc)))
      return s;
  }
  if (h->n_el[c] == 0) return DGD_OK;
  // states at this cluster's time points: its own and its coarser neighbours'
  ClusterOffsets offs;
  for (int k = 0; k < 8; ++k) offs.v[k] = k < h->nclusters ? t - h->lts_tp[k] : 0.0;
  a.elist = (const int*)h->lts_tay[c].p;
  a.nlist = h->n_tay[c];
  timed(h, 0, [&] {
    hipLaunchKernelGGL((k_taylor<N, P>), grid_of(a.nlist), block, 0, h->stream, a, offs);
  });
  // fluxes of the faces this cluster computes; integrals kept for the coarser side
  if (h->n_fl[c] > 0) {
    timed(h, 1, [&] {
      if (ivm)
        hipLaunchKernelGGL((k_face_flux<N, P, IvmLaw>), grid_of(h->n_fl[c]), block, 0, h->stream,
                           a, (const int*)h->faces.p, h->n_fl[c], (T*)h->fflux.p,
                           (const int*)h->lts_fl[c].p);
      else
        hipLaunchKernelGGL((k_face_flux<N, P, CdmLaw>), grid_of(h->n_fl[c]), block, 0, h->stream,
                           a, (const int*)h->faces.p, h->n_fl[c], (T*)h->fflux.p,
                           (const int*)h->lts_fl[c].p);
    });
  }
  if (h->n_acc[c] > 0) {
    const long long n = h->n_acc[c] * h->ref.Ns * 10;
    hipLaunchKernelGGL((k_face_accumulate<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       h->stream, h->n_acc[c], (const int*)h->lts_acc[c].p, h->ref.Ns, dtc,
                       (const T*)h->fflux.p, (T*)h->facc.p);
  }
  // volume and source terms, then the faces and the update in place
  a.elist = (const int*)h->lts_el[c].p;
  a.nlist = h->n_el[c];
  timed(h, 9, [&] { launch_volume<N, P>(h, a, ivm); });
  a.lts_c = c;
  a.facc = (T*)h->facc.p;
  a.O9 = (T*)h->U9[h->cur].p;
  a.Oa = (double*)h->Ua[h->cur].p;
  timed(h, 8, [&] {
    hipLaunchKernelGGL((k_lift_update<N, P>), grid_of(a.nlist), block, 0, h->stream, a,
                       (const int*)h->fmap.p, (const T*)h->fflux.p);
  });
  if (h->nsrc > 0) {
    // the point sources of this cluster's elements, over its step
    SrcArgs sa;
    sa.nsrc = h->nsrc;
    sa.L = h->ref.L;
    sa.elem = (const long long*)h->s_elem.p;
    sa.M6 = (const double*)h->s_M6.p;
    sa.dphi = (const double*)h->s_dphi.p;
    sa.onset = (const double*)h->s_onset.p;
    sa.param = (const double*)h->s_param.p;
    sa.rhoJ = (const double*)h->s_rhoJ.p;
    sa.kind = h->srckind;
    sa.t0 = t;
    sa.t1 = t + dtc;
    sa.ecl = (const signed char*)h->ecl.p;
    sa.only_cluster = c;
    timed(h, 2, [&] {
      hipLaunchKernelGGL((k_sources<T>), dim3(1), dim3(3 * h->ref.L), 0, h->stream, sa,
                         (T*)h->U9[h->cur].p);
    });
  }
  HIPCHK(h, hipGetLastError());
  return DGD_OK;
}

template <int N, int P> struct LtsFn {
  static dgd_status run(dgd_handle* h, long long nmacro) {
    using T = typename Prec<P>::T;
    const double mdt = h->lts_dt0 * (double)(1LL << (h->nclusters - 1));
    for (long long k = 0; k < nmacro; ++k) {
      dgd_status s = lts_advance<N, P>(h, h->nclusters - 1, h->t);
      if (s) return s;
      h->t += mdt;
      if (h->nrec > 0) {
        double* out = (double*)h->seis.p + (size_t)h->nrec_steps * h->nrec * 3;
        const int nth = h->nrec * 3;
        hipLaunchKernelGGL((k_receivers<T>), dim3((nth + 63) / 64), dim3(64), 0, h->stream, h->nrec,
                           h->ref.L, (const long long*)h->r_elem.p, (const double*)h->r_phi.p,
                           (const T*)h->U9[h->cur].p, out);
        h->nrec_steps += 1;
      }
      HIPCHK(h, hipGetLastError());
    }
    return DGD_OK;
  }
};

// dispatch on (N, precision)
template <template <int, int> class Fn, class... Args>
dgd_status dispatch(dgd_handle* h, Args... args) {
#define DGD_CASE(NN, PP) \
  if (h->N == NN && h->prec == PP) return Fn<NN, PP>::run(h, args...);
  DGD_CASE(1, 0) DGD_CASE(1, 1) DGD_CASE(1, 2)
  DGD_CASE(2, 0) DGD_CASE(2, 1) DGD_CASE(2, 2)
  DGD_CASE(3, 0) DGD_CASE(3, 1) DGD_CASE(3, 2)
  DGD_CASE(4, 0) DGD_CASE(4, 1) DGD_CASE(4, 2)
#undef DGD_CASE
  return fail(h, DGD_EINVAL, "unsupported degree/precision");
}

template <int N, int P> struct BuildFn {
  static dgd_status run(dgd_handle* h) { return build_packed<N, P>(h); }
};
template <int N, int P> struct StepFn {
  static dgd_status run(dgd_handle* h, long long n) { return step_impl<N, P>(h, n); }
};

// the predictor of the current state only (time-point states and, when the
// handle asks for them, the kept derivatives); state and time unchanged
template <int N, int P> struct PredictFn {
  static dgd_status run(dgd_handle* h) {
    const long long per = (h->ne + 7) / 8;
    StepArgs<P> a = make_args<N, P>(h);
    hipLaunchKernelGGL((k_predict<N, P>), dim3((unsigned)(8 * per)), dim3(64), 0, h->stream, a);
    HIPCHK(h, hipGetLastError());
    return DGD_OK;
  }
};

// ---------------------------------------------------------------- discrete adjoint
// The adjoint arithmetic is FP64 on FP64 handles and FP32 on the others (a
// split-BF16 handle runs its forward steps in that form and their adjoint in
// FP32, at the states of its own trajectory): mode rows of the adjoint
// states padded to the FP32/FP64 matrix-core k-step.
int adj_kpl(const dgd_handle* h) { return round_up(h->ref.L, 4); }
size_t lam_elems(const dgd_handle* h) { return (size_t)h->ne * adj_kpl(h) * 16; }

// FP32 forward operators of a split-BF16 handle (its own packs hold BF16
// hi/lo pairs), packed once beside them; the transposed adjoint operators
// come with them.
dgd_status ensure_adjoint_packs(dgd_handle* h) {
  if (h->prec != DGD_BF16 || h->Vpk32.p) return DGD_OK;
  DevBuf* fw[] = {&h->Vpk, &h->Kpk, &h->Spk, &h->Fpk, &h->Lpk, &h->Ppk, &h->KPpk};
  DevBuf* f32[] = {&h->Vpk32, &h->Kpk32, &h->Spk32, &h->Fpk32, &h->Lpk32, &h->Ppk32, &h->KPpk32};
  for (int i = 0; i < 7; ++i) std::swap(*fw[i], *f32[i]);
  const int kpl = h->kpl;
  dgd_status s = DGD_EINVAL;
  switch (h->N) {
    case 1: s = build_packed<1, PREC_F32>(h); break;
    case 2: s = build_packed<2, PREC_F32>(h); break;
    case 3: s = build_packed<3, PREC_F32>(h); break;
    case 4: s = build_packed<4, PREC_F32>(h); break;
    default: break;
  }
  h->kpl = kpl;
  for (int i = 0; i < 7; ++i) std::swap(*fw[i], *f32[i]);
  if (s) h->Vpk32.release();
  return s;
}

dgd_status alloc_adjoint(dgd_handle* h) {
  const size_t E = (size_t)h->ne, L = h->ref.L;
  dgd_status s;
  if ((s = ensure_adjoint_packs(h))) return s;
  if ((s = dalloc(h, h->lam[0], lam_elems(h) * h->tsize)) ||
      (s = dalloc(h, h->lam[1], lam_elems(h) * h->tsize)) ||
      (s = dalloc(h, h->gtr, (size_t)h->nfaces * 2 * h->ref.Nt * h->ref.Ns * 10 * h->tsize)) ||
      (s = dalloc(h, h->gmuf, (size_t)h->nfaces * 2 * sizeof(double))) ||
      (s = dalloc(h, h->lzf, lam_elems(h) * h->ref.Nt * h->tsize)) ||
      (s = dalloc(h, h->gmu, E * sizeof(double))) || (s = dalloc(h, h->gcd, E * sizeof(double))) ||
      (s = dalloc(h, h->adjW9, E * 9 * L * h->tsize)) ||
      (s = dalloc(h, h->adjWa, E * L * sizeof(double))))
    return s;
  HIPCHK(h, hipMemsetAsync(h->gmu.p, 0, E * sizeof(double), h->stream));
  HIPCHK(h, hipMemsetAsync(h->gcd.p, 0, E * sizeof(double), h->stream));
  return DGD_OK;
}

// lambda_out = (d step / d U^n)^T lambda_in at the state (U9, Ua); adds the
// material cotangents of this step to gmu, gcd
template <int N, int P>
dgd_status adjoint_step_impl(dgd_handle* h, const void* U9, const double* Ua, const void* lam_in,
                             void* lam_out, void* uz, const void* dk, const void* ak, double* gmu,
                             double* gcd) {
  using T = typename Prec<P>::T;
  using AF = typename Prec<P>::AF;
  if constexpr (P == PREC_BF16) {
    // split-BF16 forward: the adjoint arithmetic is FP32
    return adjoint_step_impl<N, PREC_F32>(h, U9, Ua, lam_in, lam_out, uz, dk, ak, gmu, gcd);
  } else {
    const long long per = (h->ne + 7) / 8;
    const dim3 grid((unsigned)(8 * per)), block(64);
    StepArgs<P> a = make_args<N, P>(h);
    if (h->prec == DGD_BF16) {
      // the FP32 operators packed beside the handle's BF16 ones; the
      // time-point states are recomputed in FP32 (uz, dk, ak are null)
      if (uz || dk || ak) return fail(h, DGD_EINVAL, "kept BF16 predictions in an FP32 adjoint");
      a.Vpk = (const AF*)h->Vpk32.p;
      a.Kpk = (const AF*)h->Kpk32.p;
      a.Spk = (const AF*)h->Spk32.p;
      a.Fpk = (const AF*)h->Fpk32.p;
      a.Lpk = (const AF*)h->Lpk32.p;
      a.Ppk = (const typename Prec<Accurate<P>::value>::AF*)h->Ppk32.p;
      a.Dkeep = nullptr;
      a.Akeep = nullptr;
    }
    a.Uz = (T*)(uz ? uz : h->Uz.p);
    a.U9 = (const T*)U9;
    a.Ua = Ua;
    a.W9 = (T*)h->adjW9.p;
    a.Wa = (double*)h->adjWa.p;
    AdjArgs<P> A;
    A.s = a;
    A.lam = (const T*)lam_in;
    A.lamOut = (T*)lam_out;
    A.gtr = (T*)h->gtr.p;
    A.gmuf = (double*)h->gmuf.p;
    A.lzf = (T*)h->lzf.p;
    A.fmap = (const int*)h->fmap.p;
    A.VTpk = (const AF*)h->VTpk.p;
    A.STpk = (const AF*)h->STpk.p;
    A.PTpk = (const AF*)h->PTpk.p;
    A.KTpk = (const AF*)h->KTpk.p;
    A.wq = (const double*)h->wqd.p;
    A.beta = (const double*)h->betad.p;
    A.Dkept = (const T*)dk;
    A.Akept = (const T*)ak;
    A.gmu = gmu ? gmu : (double*)h->gmu.p;
    A.gcd = gcd ? gcd : (double*)h->gcd.p;
    // time-point states of this step: recomputed unless the replay kept them
    if (!uz)
      timed(h, 4, [&] { hipLaunchKernelGGL((k_predict<N, P>), grid, block, 0, h->stream, a); });
    const long long fper = (h->nfaces + 7) / 8;
    timed(h, 5, [&] {
      hipLaunchKernelGGL((k_adj_face<N, P>), dim3((unsigned)(8 * fper)), block, 0, h->stream, A,
                         (const int*)h->faces.p, h->nfaces);
      hipLaunchKernelGGL((k_adj_lift<N, P>), grid, block, 0, h->stream, A);
    });
    timed(h, 6, [&] {
      if constexpr (AdjSplit<N>::value) {
        hipLaunchKernelGGL((k_adj_points<N, P>), grid, block, 0, h->stream, A);
        hipLaunchKernelGGL((k_adj_volume<N, P, false>), grid, block, 0, h->stream, A);
      } else {
        hipLaunchKernelGGL((k_adj_volume<N, P, true>), grid, block, 0, h->stream, A);
      }
    });
    HIPCHK(h, hipGetLastError());
    return DGD_OK;
  }
}

template <int N, int P> struct AdjStepFn {
  static dgd_status run(dgd_handle* h, const void* U9, const double* Ua, const void* li, void* lo,
                        void* uz, const void* dk, const void* ak, double* gmu, double* gcd) {
    return adjoint_step_impl<N, P>(h, U9, Ua, li, lo, uz, dk, ak, gmu, gcd);
  }
};

template <class T>
void launch_lam_from_f64(dgd_handle* h, const double* src, void* lam) {
  const long long n = (long long)lam_elems(h);
  hipLaunchKernelGGL((k_lam_from_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     h->stream, h->ne, h->ref.L, adj_kpl(h), src, (T*)lam);
}

template <class T>
void launch_lam_to_f64(dgd_handle* h, const void* lam, double* dst) {
  const long long n = h->ne * 10 * h->ref.L;
  hipLaunchKernelGGL((k_lam_to_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->ne, h->ref.L, adj_kpl(h), (const T*)lam, dst);
}

void release_tape(dgd_handle* h) {
  for (DevBuf& b : h->ck9) b.release();
  for (DevBuf& b : h->cka) b.release();
  h->ck9.clear();
  h->cka.clear();
  h->ck_t.clear();
  h->tape = false;
  h->tape_id = 0;
  h->tape_steps = h->tape_every = 0;
}

// Every change of the problem definition (mesh, material, law, dt, alpha_max,
// sources, receivers) drops the checkpointed run: its replay would use the new
// definition and its buffers may not match the new mesh.
void invalidate_tape(dgd_handle* h) {
  if (h->tape) (void)hipStreamSynchronize(h->stream);
  release_tape(h);
}

// The clamp alpha_max must keep the boundary moduli positive for every state:
// CDM (Eq. effective-cdb with reading R4) mu_eff = mu0 + a xi0 gamma_r -
// a gamma_r xi / 2 and lambda_eff + 2 mu_eff = lambda0 + 2 mu0 + 2 a xi0
// gamma_r - 4 a gamma_r xi / 3 are linear in a in [0, alpha_max] and in
// xi = I1/sqrt(I2) in [-sqrt 3, sqrt 3] (Cauchy-Schwarz), so their minima sit
// at the corners; IVM (Eq. ivm-model) needs alpha_max < 1 (the storage energy
// is singular at alpha = 1).
bool moduli_admissible(int law, double amax, const std::vector<double>& m, long long ne,
                       std::string* why) {
  if (law == 1) {
    if (!(amax < 1.0)) {
      *why = "alpha_max must be below 1 under the internal-variable law";
      return false;
    }
    return true;
  }
  const double r3 = std::sqrt(3.0);
  for (long long e = 0; e < ne; ++e) {
    const double lam = m[e * 8 + 1], mu = m[e * 8 + 2], gr = m[e * 8 + 3], xi0 = m[e * 8 + 4];
    for (double a : {0.0, amax})
      for (double xi : {-r3, r3}) {
        const double mue = mu + a * xi0 * gr - 0.5 * a * gr * xi;
        const double pm = lam + 2.0 * mu + 2.0 * a * xi0 * gr - 4.0 / 3.0 * a * gr * xi;
        if (!(mue > 0.0) || !(pm > 0.0)) {
          *why = "alpha_max " + std::to_string(amax) + " makes the effective moduli of element " +
                 std::to_string(e) + " non-positive";
          return false;
        }
      }
  }
  return true;
}

dgd_status copy_state(dgd_handle* h, void* d9, void* da, const void* s9, const void* sa) {
  const size_t E = (size_t)h->ne, L = h->ref.L;
  if (!d9 || !da || !s9 || !sa) return fail(h, DGD_ESTATE, "state copy between missing buffers");
  HIPCHK(h, hipMemcpyAsync(d9, s9, E * 9 * L * h->tsize, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(da, sa, E * L * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return DGD_OK;
}

// ---------------------------------------------------------------- mesh helpers
const int kFV[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};

bool inv3(const double* A, double* B, double* det) {
  // A row-major 3x3
  const double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                   A[2] * (A[3] * A[7] - A[4] * A[6]);
  *det = d;
  if (!(d > 0.0)) return false;
  const double id = 1.0 / d;
  B[0] = (A[4] * A[8] - A[5] * A[7]) * id;
  B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = (A[5] * A[6] - A[3] * A[8]) * id;
  B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = (A[3] * A[7] - A[4] * A[6]) * id;
  B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return true;
}

struct FaceKey {
  long long k[3];
  long long ef;  // element * 4 + face
  bool operator<(const FaceKey& o) const {
    if (k[0] != o.k[0]) return k[0] < o.k[0];
    if (k[1] != o.k[1]) return k[1] < o.k[1];
    if (k[2] != o.k[2]) return k[2] < o.k[2];
    return ef < o.ef;
  }
  bool same(const FaceKey& o) const { return k[0] == o.k[0] && k[1] == o.k[1] && k[2] == o.k[2]; }
};

int perm_index(const int o[3]) {
  for (int s = 0; s < 6; ++s)
    if (kPerm3[s][0] == o[0] && kPerm3[s][1] == o[1] && kPerm3[s][2] == o[2]) return s;
  return -1;
}

long long locate_point(dgd_handle* h, const double* x, double xi[3]) {
  const double tol = 1e-12;
  for (long long e = 0; e < h->ne; ++e) {
    const double* J = &h->Jinv[e * 9];
    const double* o = &h->X0[e * 3];
    double d[3] = {x[0] - o[0], x[1] - o[1], x[2] - o[2]};
    double r[3];
    for (int a = 0; a < 3; ++a) r[a] = J[a * 3] * d[0] + J[a * 3 + 1] * d[1] + J[a * 3 + 2] * d[2];
    if (r[0] >= -tol && r[1] >= -tol && r[2] >= -tol && 1.0 - r[0] - r[1] - r[2] >= -tol) {
      xi[0] = r[0];
      xi[1] = r[1];
      xi[2] = r[2];
      return e;
    }
  }
  return -1;
}

dgd_status ensure_seis(dgd_handle* h, long long extra) {
  if (h->nrec == 0) return DGD_OK;
  const long long need = h->nrec_steps + extra;
  if (need <= h->seis_cap) return DGD_OK;
  long long cap = std::max<long long>(need, std::max<long long>(1024, 2 * h->seis_cap));
  void* p = nullptr;
  HIPCHK(h, hipMalloc(&p, (size_t)cap * h->nrec * 3 * sizeof(double)));
  if (h->seis.p && h->nrec_steps > 0)
    HIPCHK(h, hipMemcpyAsync(p, h->seis.p, (size_t)h->nrec_steps * h->nrec * 3 * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->seis.release();
  h->seis.p = p;
  h->seis.n = (size_t)cap * h->nrec * 3 * sizeof(double);
  h->seis_cap = cap;
  return DGD_OK;
}

// bytes of the time-point states of all elements, [E][Nt][L][10], and of the
// zeroed tail after them that the matrix cores' in-place reads of the last
// element's padding rows reach (KPL * 16 entries)
size_t uz_bytes(const dgd_handle* h) {
  return (size_t)h->ne * h->ref.Nt * h->ref.L * 10 * h->tsize;
}
size_t uz_tail(const dgd_handle* h) { return (size_t)h->kpl * 16 * h->tsize; }

// a buffer of `slots` consecutive time-point-state arrays and the zeroed tail
dgd_status alloc_uz(dgd_handle* h, DevBuf& b, size_t slots) {
  dgd_status s = dalloc(h, b, slots * uz_bytes(h) + uz_tail(h));
  if (s) return s;
  HIPCHK(h, hipMemsetAsync(b.p, 0, b.n, h->stream));
  return DGD_OK;
}

dgd_status alloc_state(dgd_handle* h) {
  const size_t L = h->ref.L, E = (size_t)h->ne;
  dgd_status s;
  for (int i = 0; i < 2; ++i) {
    if ((s = dalloc(h, h->U9[i], E * 9 * L * h->tsize))) return s;
    if ((s = dalloc(h, h->Ua[i], E * L * sizeof(double)))) return s;
  }
  if ((s = alloc_uz(h, h->Uz, 1))) return s;
  if ((s = dalloc(h, h->fflux, (size_t)h->nfaces * h->ref.Ns * 10 * h->tsize))) return s;
  if ((s = dalloc(h, h->flag, sizeof(int)))) return s;
  HIPCHK(h, hipMemsetAsync(h->flag.p, 0, sizeof(int), h->stream));
  return DGD_OK;
}

template <class T>
void launch_from_f64(dgd_handle* h, const double* src) {
  const long long n = h->ne * 10 * h->ref.L;
  hipLaunchKernelGGL((k_from_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->ne, h->ref.L, src, (T*)h->U9[h->cur].p, (double*)h->Ua[h->cur].p);
}

template <class T>
void launch_to_f64(dgd_handle* h, double* dst) {
  const long long n = h->ne * 10 * h->ref.L;
  hipLaunchKernelGGL((k_to_f64<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->ne, h->ref.L, (const T*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                     dst);
}

}  // namespace

// ================================================================== C interface
extern "C" {

dgd_status dgd_create(int N, int precision, void* hip_stream, dgd_handle** out) {
  if (!out) return DGD_EINVAL;
  *out = nullptr;
  if (N < 1 || N > 4 || precision < 0 || precision > 2) return DGD_EINVAL;
  dgd_handle* h = new (std::nothrow) dgd_handle();
  if (!h) return DGD_ENOMEM;
  h->N = N;
  h->prec = precision;
  h->stream = (hipStream_t)hip_stream;
  h->tsize = precision == DGD_FP64 ? 8 : 4;
  // volume terms three elements per wavefront where that measured faster
  // (FP32 at degree 4: 118 against 133 ms per step on 5,308,416 tets; slower
  // in FP64 and with the split BF16 operands)
  h->vol3 = precision == DGD_FP32 && N == 4;
  if (hipGetDevice(&h->device) != hipSuccess ||
      scratch_address(h->device, &h->noalloc_part) != hipSuccess) {
    delete h;
    return DGD_EDEVICE;
  }
  try {
    h->ref = build_reference(N);
  } catch (...) {
    delete h;
    return DGD_EINVAL;
  }
  double ws = 0.0;
  for (double w : h->ref.wq) ws += w;
  h->inv_wsum = 1.0 / ws;
  // cell mean of phi_0 over the reference tetrahedron: 6 * int phi_0
  double m0 = 0.0;
  for (int q = 0; q < h->ref.Q; ++q) m0 += h->ref.wq[q] * h->ref.V[(size_t)q * h->ref.L];
  h->phi0_mean = 6.0 * m0;
  dgd_status s = dispatch<BuildFn>(h);
  if (s == DGD_OK) s = upload(h, h->Vd, h->ref.V);
  if (s == DGD_OK) s = upload(h, h->wqd, h->ref.wq);
  if (s == DGD_OK) s = upload(h, h->Pwd, h->ref.Pw);
  if (s == DGD_OK) s = upload(h, h->betad, h->ref.beta);
  if (s != DGD_OK) {
    delete h;
    return s;
  }
  *out = h;
  return DGD_OK;
}

dgd_status dgd_destroy(dgd_handle* h) {
  if (h) {
    (void)hipStreamSynchronize(h->stream);
    delete h;
  }
  return DGD_OK;
}

const char* dgd_last_error(const dgd_handle* h) { return h ? h->err.c_str() : "null handle"; }

dgd_status dgd_sizes(const dgd_handle* h, int* L, int* Q, int* Ns, int* Nt) {
  if (!h) return DGD_EINVAL;
  if (L) *L = h->ref.L;
  if (Q) *Q = h->ref.Q;
  if (Ns) *Ns = h->ref.Ns;
  if (Nt) *Nt = h->ref.Nt;
  return DGD_OK;
}

dgd_status dgd_set_mesh(dgd_handle* h, int64_t nv, const double* xyz, int64_t ne,
                        const int64_t* tets, const int8_t* face_tag, const int64_t* pmap) {
  if (!h) return DGD_EINVAL;
  if (nv <= 0 || ne <= 0 || !xyz || !tets || !face_tag) return fail(h, DGD_EINVAL, "bad mesh arguments");
  if (ne > (1LL << 30)) return fail(h, DGD_EINVAL, "too many elements");
  invalidate_tape(h);
  h->have_mesh = h->have_state = false;
  std::vector<long long> ids((size_t)ne * 4);
  for (long long i = 0; i < ne * 4; ++i) {
    const long long v = tets[i];
    if (v < 0 || v >= nv) return fail(h, DGD_EINVAL, "vertex id out of range");
    long long g = v;
    if (pmap) {
      g = pmap[v];
      if (g < 0 || g >= nv) return fail(h, DGD_EINVAL, "periodic map out of range");
    }
    ids[i] = g;
  }
  h->ne = ne;
  h->X0.assign((size_t)ne * 3, 0.0);
  h->Jinv.assign((size_t)ne * 9, 0.0);
  h->detJ.assign((size_t)ne, 0.0);
  std::vector<double> geo((size_t)ne * 16, 0.0), fgeo((size_t)ne * 16, 0.0);
  for (long long e = 0; e < ne; ++e) {
    const double* x[4];
    for (int k = 0; k < 4; ++k) x[k] = xyz + 3 * tets[e * 4 + k];
    double J[9];  // J[d][e] = x_{e+1,d} - x_{0,d}
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) J[d * 3 + c] = x[c + 1][d] - x[0][d];
    double det;
    if (!inv3(J, &h->Jinv[e * 9], &det))
      return fail(h, DGD_EINVAL, "inverted or degenerate tetrahedron " + std::to_string(e));
    h->detJ[e] = det;
    for (int d = 0; d < 3; ++d) h->X0[e * 3 + d] = x[0][d];
    for (int k = 0; k < 9; ++k) geo[e * 16 + k] = h->Jinv[e * 9 + k];
    geo[e * 16 + 9] = det;
    for (int f = 0; f < 4; ++f) {
      const double* A = x[kFV[f][0]];
      const double* B = x[kFV[f][1]];
      const double* C = x[kFV[f][2]];
      double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
      const double ln = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int d = 0; d < 3; ++d) fgeo[(e * 4 + f) * 4 + d] = cr[d] / ln;
      fgeo[(e * 4 + f) * 4 + 3] = 0.5 * ln / det;
    }
  }
  // connectivity
  std::vector<int> conn((size_t)ne * 8, 0);
  std::vector<FaceKey> keys;
  keys.reserve((size_t)ne * 4);
  for (long long e = 0; e < ne; ++e)
    for (int f = 0; f < 4; ++f) {
      const int tag = face_tag[e * 4 + f];
      long long g[3];
      for (int j = 0; j < 3; ++j) g[j] = ids[e * 4 + kFV[f][j]];
      if (g[0] == g[1] || g[0] == g[2] || g[1] == g[2])
        return fail(h, DGD_EINVAL, "face with repeated vertices");
      int order[3] = {0, 1, 2};
      std::sort(order, order + 3, [&](int a, int b) { return g[a] < g[b]; });
      const int sp = perm_index(order);
      int kind;
      if (tag == DGD_FACE_INTERIOR) {
        kind = 0;
        FaceKey k;
        for (int j = 0; j < 3; ++j) k.k[j] = g[order[j]];
        k.ef = e * 4 + f;
        keys.push_back(k);
      } else if (tag == DGD_BC_FREE) {
        kind = 1;
      } else if (tag == DGD_BC_ABSORB) {
        kind = 2;
      } else {
        return fail(h, DGD_EINVAL, "bad face tag");
      }
      conn[(e * 4 + f) * 2] = -1;
      conn[(e * 4 + f) * 2 + 1] = kind | (sp << 2);
    }
  std::sort(keys.begin(), keys.end());
  for (size_t i = 0; i < keys.size();) {
    if (i + 1 >= keys.size() || !keys[i].same(keys[i + 1]) ||
        (i + 2 < keys.size() && keys[i].same(keys[i + 2])))
      return fail(h, DGD_EINVAL, "interior face without exactly one partner");
    const long long a = keys[i].ef, b = keys[i + 1].ef;
    for (int side = 0; side < 2; ++side) {
      const long long me = side ? b : a, ot = side ? a : b;
      int& w = conn[(me)*2 + 1];
      const int sq = conn_perm(conn[ot * 2 + 1]);
      w |= ((int)(ot % 4) << 5) | (sq << 7);
      conn[me * 2] = (int)(ot / 4);
    }
    i += 2;
  }
  // face list: every interior face once (first side = the lower element*4+face),
  // every boundary face once; faces follow their first element's order
  std::vector<int> faces, fmap((size_t)ne * 4, -1);
  faces.reserve((size_t)ne * 4);
  long long nfaces = 0;
  for (long long ef = 0; ef < ne * 4; ++ef) {
    const int kind = conn_kind(conn[ef * 2 + 1]);
    if (kind != 0) {
      faces.push_back((int)ef);
      faces.push_back(-1);
      fmap[ef] = (int)(nfaces * 2);
      ++nfaces;
    } else {
      const long long of = (long long)conn[ef * 2] * 4 + conn_nface(conn[ef * 2 + 1]);
      if (of > ef) {
        faces.push_back((int)ef);
        faces.push_back((int)of);
        fmap[ef] = (int)(nfaces * 2);
        fmap[of] = (int)(nfaces * 2 + 1);
        ++nfaces;
      } else if (of == ef) {
        return fail(h, DGD_EINVAL, "face matched with itself");
      }
    }
  }
  if (nfaces * 2 > (long long)INT32_MAX) return fail(h, DGD_EINVAL, "too many faces");
  for (long long ef = 0; ef < ne * 4; ++ef)
    if (fmap[ef] < 0) return fail(h, DGD_EINVAL, "face without a face record");
  dgd_status s;
  if ((s = upload(h, h->geo, geo)) || (s = upload(h, h->fgeo, fgeo)) || (s = upload(h, h->conn, conn)) ||
      (s = upload(h, h->faces, faces)) || (s = upload(h, h->fmap, fmap)))
    return s;
  h->nfaces = nfaces;
  h->fgeo_h = fgeo;
  h->nbr_h.assign((size_t)ne * 4, -1);
  for (long long ef = 0; ef < ne * 4; ++ef)
    if (conn_kind(conn[ef * 2 + 1]) == 0) h->nbr_h[ef] = conn[ef * 2];
  h->faces_h.swap(faces);
  h->nclusters = 0;
  h->cl_h.clear();
  if ((s = alloc_state(h))) return s;
  h->have_mesh = true;
  h->have_mat = false;
  h->nsrc = 0;
  h->nrec = 0;
  h->nrec_steps = 0;
  return DGD_OK;
}

dgd_status dgd_set_material(dgd_handle* h, const double* rho, const double* lambda0,
                            const double* mu0, const double* gamma_r, const double* xi0,
                            const double* Cd) {
  if (!h) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  if (!rho || !lambda0 || !mu0 || !gamma_r || !xi0 || !Cd) return fail(h, DGD_EINVAL, "null array");
  std::vector<double> m((size_t)h->ne * 8, 0.0);
  for (long long e = 0; e < h->ne; ++e) {
    if (!(rho[e] > 0.0) || !(mu0[e] > 0.0)) return fail(h, DGD_EINVAL, "rho and mu0 must be positive");
    m[e * 8 + 0] = rho[e];
    m[e * 8 + 1] = lambda0[e];
    m[e * 8 + 2] = mu0[e];
    m[e * 8 + 3] = gamma_r[e];
    m[e * 8 + 4] = xi0[e];
    m[e * 8 + 5] = Cd[e];
  }
  std::string why;
  if (h->have_params && !moduli_admissible(0, h->amax, m, h->ne, &why))
    return fail(h, DGD_EINVAL, why);
  invalidate_tape(h);
  dgd_status s = upload(h, h->mat, m);
  if (s) return s;
  h->rho_h.assign(rho, rho + h->ne);
  h->mat_h.swap(m);
  h->law = 0;
  h->have_mat = true;
  return DGD_OK;
}

dgd_status dgd_set_material_ivm(dgd_handle* h, const double* rho, const double* lambda0,
                                const double* mu0, const double* gamma_b, const double* tau_b) {
  if (!h) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  if (!rho || !lambda0 || !mu0 || !gamma_b || !tau_b) return fail(h, DGD_EINVAL, "null array");
  std::vector<double> m((size_t)h->ne * 8, 0.0);
  for (long long e = 0; e < h->ne; ++e) {
    if (!(rho[e] > 0.0) || !(mu0[e] > 0.0)) return fail(h, DGD_EINVAL, "rho and mu0 must be positive");
    if (!(gamma_b[e] > 0.0) || !(tau_b[e] > 0.0))
      return fail(h, DGD_EINVAL, "gamma_b and tau_b must be positive");
    m[e * 8 + 0] = rho[e];
    m[e * 8 + 1] = lambda0[e];
    m[e * 8 + 2] = mu0[e];
    m[e * 8 + 3] = gamma_b[e];
    m[e * 8 + 5] = 1.0 / (gamma_b[e] * tau_b[e]);
  }
  std::string why;
  if (h->have_params && !moduli_admissible(1, h->amax, m, h->ne, &why))
    return fail(h, DGD_EINVAL, why);
  invalidate_tape(h);
  dgd_status s = upload(h, h->mat, m);
  if (s) return s;
  h->rho_h.assign(rho, rho + h->ne);
  h->mat_h.swap(m);
  h->law = 1;
  h->have_mat = true;
  return DGD_OK;
}

dgd_status dgd_set_params(dgd_handle* h, double dt, double alpha_max) {
  if (!h) return DGD_EINVAL;
  if (!(dt > 0.0) || !(alpha_max >= 0.0)) return fail(h, DGD_EINVAL, "dt > 0 and alpha_max >= 0 needed");
  std::string why;
  if (h->have_mat && !moduli_admissible(h->law, alpha_max, h->mat_h, h->ne, &why))
    return fail(h, DGD_EINVAL, why);
  invalidate_tape(h);
  h->dt = dt;
  h->amax = alpha_max;
  h->have_params = true;
  return DGD_OK;
}

dgd_status dgd_get_quadrature_points(dgd_handle* h, int64_t e0, int64_t count, double* xyz) {
  if (!h || !xyz) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  if (e0 < 0 || count < 0 || e0 + count > h->ne) return fail(h, DGD_EINVAL, "element range");
  const int Q = h->ref.Q;
  xyz -= (size_t)e0 * Q * 3;
  for (long long e = e0; e < e0 + count; ++e) {
    // x = X0 + J xi, J = inverse of Jinv (recompute from Jinv for independence of storage)
    double J[9], det;
    inv3(&h->Jinv[e * 9], J, &det);
    for (int q = 0; q < Q; ++q) {
      const double* xi = &h->ref.xq[3 * q];
      for (int d = 0; d < 3; ++d)
        xyz[(e * Q + q) * 3 + d] =
            h->X0[e * 3 + d] + J[d * 3] * xi[0] + J[d * 3 + 1] * xi[1] + J[d * 3 + 2] * xi[2];
    }
  }
  return DGD_OK;
}

dgd_status dgd_set_state_from_points(dgd_handle* h, int64_t e0, int64_t count,
                                     const double* vals) {
  if (!h || !vals) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  if (e0 < 0 || count <= 0 || e0 + count > h->ne) return fail(h, DGD_EINVAL, "element range");
  const size_t n = (size_t)count * h->ref.Q * 10;
  dgd_status s = dalloc(h, h->tmp, n * sizeof(double));
  if (s) return s;
  HIPCHK(h, hipMemcpyAsync(h->tmp.p, vals, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  const long long nt = count * 10 * h->ref.L;
  const dim3 g((unsigned)((nt + 255) / 256)), b(256);
  const size_t L = h->ref.L;
  if (h->prec == DGD_FP64)
    hipLaunchKernelGGL((k_project<double>), g, b, 0, h->stream, (long long)count, h->ref.L,
                       h->ref.Q, (const double*)h->Pwd.p, (const double*)h->tmp.p,
                       (double*)h->U9[h->cur].p + (size_t)e0 * 9 * L,
                       (double*)h->Ua[h->cur].p + (size_t)e0 * L);
  else
    hipLaunchKernelGGL((k_project<float>), g, b, 0, h->stream, (long long)count, h->ref.L,
                       h->ref.Q, (const double*)h->Pwd.p, (const double*)h->tmp.p,
                       (float*)h->U9[h->cur].p + (size_t)e0 * 9 * L,
                       (double*)h->Ua[h->cur].p + (size_t)e0 * L);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->tmp.release();
  h->have_state = true;
  h->t = 0.0;
  return DGD_OK;
}

dgd_status dgd_set_state(dgd_handle* h, const double* dofs, int on_device) {
  if (!h || !dofs) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  const size_t n = (size_t)h->ne * 10 * h->ref.L;
  const double* src = dofs;
  if (!on_device) {
    dgd_status s = dalloc(h, h->tmp, n * sizeof(double));
    if (s) return s;
    HIPCHK(h, hipMemcpyAsync(h->tmp.p, dofs, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    src = (const double*)h->tmp.p;
  }
  if (h->prec == DGD_FP64)
    launch_from_f64<double>(h, src);
  else
    launch_from_f64<float>(h, src);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!on_device) h->tmp.release();
  h->have_state = true;
  h->t = 0.0;
  return DGD_OK;
}

dgd_status dgd_get_state(dgd_handle* h, double* dofs, int on_device) {
  if (!h || !dofs) return DGD_EINVAL;
  if (!h->have_state) return fail(h, DGD_ESTATE, "no state");
  const size_t n = (size_t)h->ne * 10 * h->ref.L;
  double* dst = dofs;
  if (!on_device) {
    dgd_status s = dalloc(h, h->tmp, n * sizeof(double));
    if (s) return s;
    dst = (double*)h->tmp.p;
  }
  if (h->prec == DGD_FP64)
    launch_to_f64<double>(h, dst);
  else
    launch_to_f64<float>(h, dst);
  HIPCHK(h, hipGetLastError());
  if (!on_device) {
    HIPCHK(h, hipMemcpyAsync(dofs, dst, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!on_device) h->tmp.release();
  return DGD_OK;
}

dgd_status dgd_get_point_values(dgd_handle* h, int64_t e0, int64_t count, double* vals,
                                int on_device) {
  if (!h || !vals) return DGD_EINVAL;
  if (!h->have_state) return fail(h, DGD_ESTATE, "no state");
  if (e0 < 0 || count <= 0 || e0 + count > h->ne) return fail(h, DGD_EINVAL, "element range");
  const size_t L = h->ref.L, Q = h->ref.Q, n = (size_t)count * Q * 10;
  double* dst = vals;
  if (!on_device) {
    dgd_status s = dalloc(h, h->tmp, n * sizeof(double));
    if (s) return s;
    dst = (double*)h->tmp.p;
  }
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (h->prec == DGD_FP64)
    hipLaunchKernelGGL((k_point_values<double>), g, b, 0, h->stream, (long long)count, (int)L,
                       (int)Q, (const double*)h->Vd.p, (const double*)h->U9[h->cur].p + e0 * 9 * L,
                       (const double*)h->Ua[h->cur].p + e0 * L, dst);
  else
    hipLaunchKernelGGL((k_point_values<float>), g, b, 0, h->stream, (long long)count, (int)L,
                       (int)Q, (const double*)h->Vd.p, (const float*)h->U9[h->cur].p + e0 * 9 * L,
                       (const double*)h->Ua[h->cur].p + e0 * L, dst);
  HIPCHK(h, hipGetLastError());
  if (!on_device)
    HIPCHK(h, hipMemcpyAsync(vals, dst, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!on_device) h->tmp.release();
  return DGD_OK;
}

dgd_status dgd_set_time(dgd_handle* h, double t) {
  if (!h) return DGD_EINVAL;
  h->t = t;
  return DGD_OK;
}

dgd_status dgd_get_time(const dgd_handle* h, double* t) {
  if (!h || !t) return DGD_EINVAL;
  *t = h->t;
  return DGD_OK;
}

dgd_status dgd_set_predictor(dgd_handle* h, int kind, int iterations) {
  if (!h) return DGD_EINVAL;
  if ((kind != DGD_PREDICT_CK && kind != DGD_PREDICT_PICARD) || iterations < 0)
    return fail(h, DGD_EINVAL, "predictor kind 0 or 1 and iterations >= 0 needed");
  invalidate_tape(h);
  h->predictor = kind;
  h->picard_iters = iterations;
  return DGD_OK;
}

dgd_status dgd_set_clusters(dgd_handle* h, const int32_t* cluster, double dt0) {
  if (!h) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  invalidate_tape(h);
  for (auto* v : {&h->lts_el, &h->lts_tay, &h->lts_fl, &h->lts_acc})
    for (DevBuf& b : *v) b.release();
  h->nclusters = 0;
  h->cl_h.clear();
  if (!cluster) return DGD_OK;
  if (!(dt0 > 0.0)) return fail(h, DGD_EINVAL, "dt0 > 0 needed");
  const long long ne = h->ne;
  std::vector<signed char> cl((size_t)ne);
  int C = 0;
  for (long long e = 0; e < ne; ++e) {
    if (cluster[e] < 0 || cluster[e] > 7) return fail(h, DGD_EINVAL, "clusters 0..7");
    cl[e] = (signed char)cluster[e];
    C = std::max(C, (int)cluster[e] + 1);
  }
  for (long long ef = 0; ef < ne * 4; ++ef) {
    const int nb = h->nbr_h[ef];
    if (nb >= 0 && std::abs((int)cl[ef / 4] - (int)cl[nb]) > 1)
      return fail(h, DGD_EINVAL, "face neighbours more than one cluster apart");
  }
  std::vector<std::vector<int>> el(C), tay(C), fl(C), acc(C);
  for (long long e = 0; e < ne; ++e) el[cl[e]].push_back((int)e);
  for (int c = 0; c < C; ++c) {
    tay[c] = el[c];
    if (c + 1 < C) {
      std::vector<int> extra;
      for (int e : el[c + 1])
        for (int f = 0; f < 4; ++f) {
          const int nb = h->nbr_h[(size_t)e * 4 + f];
          if (nb >= 0 && cl[nb] == c) {
            extra.push_back(e);
            break;
          }
        }
      tay[c].insert(tay[c].end(), extra.begin(), extra.end());
      std::sort(tay[c].begin(), tay[c].end());
    }
  }
  for (long long fid = 0; fid < h->nfaces; ++fid) {
    const int ef = h->faces_h[fid * 2], of = h->faces_h[fid * 2 + 1];
    const int c1 = cl[ef >> 2];
    if (of < 0) {
      fl[c1].push_back((int)fid);
      continue;
    }
    const int c2 = cl[of >> 2], cm = std::min(c1, c2);
    fl[cm].push_back((int)fid);
    if (c1 != c2) acc[cm].push_back((int)fid);
  }
  h->lts_el.resize(C);
  h->lts_tay.resize(C);
  h->lts_fl.resize(C);
  h->lts_acc.resize(C);
  h->n_el.assign(C, 0);
  h->n_tay.assign(C, 0);
  h->n_fl.assign(C, 0);
  h->n_acc.assign(C, 0);
  dgd_status s;
  for (int c = 0; c < C; ++c) {
    if ((s = upload(h, h->lts_el[c], el[c])) || (s = upload(h, h->lts_tay[c], tay[c])) ||
        (s = upload(h, h->lts_fl[c], fl[c])) || (s = upload(h, h->lts_acc[c], acc[c])))
      return s;
    h->n_el[c] = (long long)el[c].size();
    h->n_tay[c] = (long long)tay[c].size();
    h->n_fl[c] = (long long)fl[c].size();
    h->n_acc[c] = (long long)acc[c].size();
  }
  if ((s = upload(h, h->ecl, cl))) return s;
  h->cl_h.swap(cl);
  h->nclusters = C;
  h->lts_dt0 = dt0;
  return DGD_OK;
}

dgd_status dgd_make_clusters(dgd_handle* h, double cfl, int max_clusters, int32_t* cluster,
                             double* dt0) {
  if (!h || !cluster || !dt0) return DGD_EINVAL;
  if (!h->have_mesh || !h->have_mat) return fail(h, DGD_ESTATE, "mesh and material first");
  if (!(cfl > 0.0) || max_clusters < 1 || max_clusters > 8)
    return fail(h, DGD_EINVAL, "cfl > 0 and 1..8 clusters needed");
  const long long ne = h->ne;
  // admissible step of every element: cfl 2 r_in / ((2N+1) c_p), r_in = 3 V / A
  std::vector<double> dte((size_t)ne);
  double dmin = 1e300;
  for (long long e = 0; e < ne; ++e) {
    const double* m = &h->mat_h[e * 8];
    const double cp = std::sqrt((m[1] + 2.0 * m[2]) / m[0]);   // intact moduli
    // |S_f| / |J| are kept per face; V = |J| / 6, so r_in = 3 V / A = 1 / (2 sum |S_f|/|J|)
    double sa = 0.0;
    for (int f = 0; f < 4; ++f) sa += h->fgeo_h[(e * 4 + f) * 4 + 3];
    const double r_in = 1.0 / (2.0 * sa);
    dte[e] = cfl * 2.0 * r_in / ((2 * h->N + 1) * cp);
    dmin = std::min(dmin, dte[e]);
  }
  std::vector<int> c((size_t)ne);
  for (long long e = 0; e < ne; ++e)
    c[e] = std::max(0, std::min(max_clusters - 1, (int)std::floor(std::log2(dte[e] / dmin) + 1e-12)));
  for (bool changed = true; changed;) {
    changed = false;
    for (long long e = 0; e < ne; ++e)
      for (int f = 0; f < 4; ++f) {
        const int nb = h->nbr_h[(size_t)e * 4 + f];
        if (nb >= 0 && c[e] > c[nb] + 1) {
          c[e] = c[nb] + 1;
          changed = true;
        }
      }
  }
  for (long long e = 0; e < ne; ++e) cluster[e] = c[e];
  *dt0 = dmin;
  return DGD_OK;
}

dgd_status dgd_step_lts(dgd_handle* h, int64_t nmacro) {
  if (!h) return DGD_EINVAL;
  if (nmacro < 0) return fail(h, DGD_EINVAL, "negative step count");
  if (h->nclusters < 1) return fail(h, DGD_ESTATE, "dgd_set_clusters first");
  if (!h->have_mesh || !h->have_mat || !h->have_params || !h->have_state)
    return fail(h, DGD_ESTATE, "mesh, material, params and state are needed before step");
  if (h->predictor != 0)
    return fail(h, DGD_EINVAL, "local time stepping uses the Cauchy-Kovalevskaya predictor");
  const size_t E = (size_t)h->ne;
  dgd_status s;
  if ((s = dalloc(h, h->Dall, E * h->N * h->kpl * 16 * h->tsize))) return s;
  if (h->facc.n != (size_t)h->nfaces * h->ref.Ns * 10 * h->tsize) {
    if ((s = dalloc(h, h->facc, (size_t)h->nfaces * h->ref.Ns * 10 * h->tsize))) return s;
    HIPCHK(h, hipMemsetAsync(h->facc.p, 0, h->facc.n, h->stream));
  }
  if ((s = ensure_seis(h, nmacro))) return s;
  if ((s = dispatch<LtsFn>(h, (long long)nmacro))) return s;
  return dgd_synchronize(h);
}

dgd_status dgd_set_point_sources(dgd_handle* h, int n, const double* xyz, const double* M6,
                                 const double* t_onset, const double* stf_param, int stf_kind) {
  if (!h) return DGD_EINVAL;
  if (!h->have_mesh || !h->have_mat) return fail(h, DGD_ESTATE, "mesh and material first");
  if (n < 0 || (n > 0 && (!xyz || !M6 || !t_onset || !stf_param)))
    return fail(h, DGD_EINVAL, "bad source arguments");
  if (stf_kind != DGD_STF_RICKER && stf_kind != DGD_STF_GAUSSIAN)
    return fail(h, DGD_EINVAL, "bad source time function");
  invalidate_tape(h);
  const int L = h->ref.L;
  std::vector<long long> elem(n);
  std::vector<double> dphi((size_t)n * 3 * L), rhoJ(n), m6(M6, M6 + 6 * (size_t)n),
      on(t_onset, t_onset + n), par(stf_param, stf_param + n);
  std::vector<double> phi(L), dxi(3 * L);
  for (int k = 0; k < n; ++k) {
    double xi[3];
    const long long e = locate_point(h, xyz + 3 * k, xi);
    if (e < 0) return fail(h, DGD_EINVAL, "source outside the mesh");
    if (!(par[k] > 0.0)) return fail(h, DGD_EINVAL, "stf parameter must be positive");
    elem[k] = e;
    basis_eval(h->N, xi, phi.data(), dxi.data());
    const double* Ji = &h->Jinv[e * 9];
    for (int d = 0; d < 3; ++d)
      for (int l = 0; l < L; ++l) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += dxi[a * L + l] * Ji[a * 3 + d];
        dphi[((size_t)k * 3 + d) * L + l] = s;
      }
    rhoJ[k] = h->rho_h[e] * h->detJ[e];
  }
  dgd_status s;
  if ((s = upload(h, h->s_elem, elem)) || (s = upload(h, h->s_M6, m6)) ||
      (s = upload(h, h->s_dphi, dphi)) || (s = upload(h, h->s_onset, on)) ||
      (s = upload(h, h->s_param, par)) || (s = upload(h, h->s_rhoJ, rhoJ)))
    return s;
  h->nsrc = n;
  h->srckind = stf_kind;
  return DGD_OK;
}

dgd_status dgd_set_receivers(dgd_handle* h, int nrec, const double* xyz) {
  if (!h) return DGD_EINVAL;
  if (!h->have_mesh) return fail(h, DGD_ESTATE, "set_mesh first");
  if (nrec < 0 || (nrec > 0 && !xyz)) return fail(h, DGD_EINVAL, "bad receiver arguments");
  invalidate_tape(h);
  const int L = h->ref.L;
  std::vector<long long> elem(nrec);
  std::vector<double> phi((size_t)nrec * L);
  for (int r = 0; r < nrec; ++r) {
    double xi[3];
    const long long e = locate_point(h, xyz + 3 * r, xi);
    if (e < 0) return fail(h, DGD_EINVAL, "receiver outside the mesh");
    elem[r] = e;
    basis_eval(h->N, xi, &phi[(size_t)r * L], nullptr);
  }
  dgd_status s;
  if ((s = upload(h, h->r_elem, elem)) || (s = upload(h, h->r_phi, phi))) return s;
  h->nrec = nrec;
  h->nrec_steps = 0;
  h->seis.release();
  h->seis_cap = 0;
  return DGD_OK;
}

dgd_status dgd_set_check_interval(dgd_handle* h, int64_t every) {
  if (!h || every < 1) return DGD_EINVAL;
  h->check_every = every;
  return DGD_OK;
}

dgd_status dgd_synchronize(dgd_handle* h) {
  if (!h) return DGD_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->flag.p) {
    int f = 0;
    HIPCHK(h, hipMemcpy(&f, h->flag.p, sizeof(int), hipMemcpyDeviceToHost));
    if (f) return fail(h, DGD_ENUMERIC, "non-finite value in the state");
  }
  return DGD_OK;
}

dgd_status dgd_step(dgd_handle* h, int64_t nsteps) {
  if (!h) return DGD_EINVAL;
  if (nsteps < 0) return fail(h, DGD_EINVAL, "negative step count");
  if (!h->have_mesh || !h->have_mat || !h->have_params || !h->have_state)
    return fail(h, DGD_ESTATE, "mesh, material, params and state are needed before step");
  dgd_status s = ensure_seis(h, nsteps);
  if (s) return s;
  long long left = nsteps;
  while (left > 0) {
    long long chunk = std::min<long long>(left, h->check_every - h->steps_since_check);
    if (chunk <= 0) chunk = 1;
    if ((s = dispatch<StepFn>(h, chunk))) return s;
    left -= chunk;
    h->steps_since_check += chunk;
    if (h->steps_since_check >= h->check_every) {
      h->steps_since_check = 0;
      if ((s = dgd_synchronize(h))) return s;
    }
  }
  return DGD_OK;
}

dgd_status dgd_num_seismogram_steps(const dgd_handle* h, int64_t* n) {
  if (!h || !n) return DGD_EINVAL;
  *n = h->nrec_steps;
  return DGD_OK;
}

dgd_status dgd_get_seismograms(dgd_handle* h, double* out, int64_t* nrecorded) {
  if (!h) return DGD_EINVAL;
  if (nrecorded) *nrecorded = h->nrec_steps;
  if (h->nrec == 0 || h->nrec_steps == 0) return DGD_OK;
  if (!out) return fail(h, DGD_EINVAL, "null output");
  HIPCHK(h, hipMemcpyAsync(out, h->seis.p, (size_t)h->nrec_steps * h->nrec * 3 * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DGD_OK;
}

dgd_status dgd_clear_seismograms(dgd_handle* h) {
  if (!h) return DGD_EINVAL;
  h->nrec_steps = 0;
  return DGD_OK;
}

dgd_status dgd_energy(dgd_handle* h, double* E) {
  if (!h || !E) return DGD_EINVAL;
  if (!h->have_state || !h->have_mat || !h->have_params)
    return fail(h, DGD_ESTATE, "state, material and params needed");
  if (h->law != 0) return fail(h, DGD_EINVAL, "the energy is that of the continuum-damage law");
  dgd_status s = dalloc(h, h->tmp, (size_t)(h->ne + 1) * sizeof(double));
  if (s) return s;
  double* part = (double*)h->tmp.p;
  if (h->prec == DGD_FP64)
    hipLaunchKernelGGL((k_energy<double>), dim3((unsigned)h->ne), dim3(64), 0, h->stream, h->ne,
                       h->ref.L, h->ref.Q, (const double*)h->Vd.p, (const double*)h->wqd.p,
                       (const double*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                       (const double*)h->geo.p, (const double*)h->mat.p, h->amax, 1e-15, part);
  else
    hipLaunchKernelGGL((k_energy<float>), dim3((unsigned)h->ne), dim3(64), 0, h->stream, h->ne,
                       h->ref.L, h->ref.Q, (const double*)h->Vd.p, (const double*)h->wqd.p,
                       (const float*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                       (const double*)h->geo.p, (const double*)h->mat.p, h->amax, 1e-15, part);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, h->stream, h->ne, part, part + h->ne);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(E, part + h->ne, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->tmp.release();
  return DGD_OK;
}

dgd_status dgd_energy_noalloc(dgd_handle* h, double* E) {
  if (!h || !E) return DGD_EINVAL;
  if (h->ne > kNoallocMaxElems)
    return fail(h, DGD_EINVAL,
                "dgd_energy_noalloc takes at most " + std::to_string(kNoallocMaxElems) +
                    " elements (its static partial-sum buffer); this mesh has " +
                    std::to_string(h->ne) + ": use dgd_energy");
  if (!h->have_state || !h->have_mat || !h->have_params)
    return fail(h, DGD_ESTATE, "state, material and params needed");
  if (h->law != 0) return fail(h, DGD_EINVAL, "the energy is that of the continuum-damage law");
  double* part = h->noalloc_part;   // every entry [0, ne) is written before it is read
  if (h->prec == DGD_FP64)
    hipLaunchKernelGGL((k_energy<double>), dim3((unsigned)h->ne), dim3(64), 0, h->stream, h->ne,
                       h->ref.L, h->ref.Q, (const double*)h->Vd.p, (const double*)h->wqd.p,
                       (const double*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                       (const double*)h->geo.p, (const double*)h->mat.p, h->amax, 1e-15, part);
  else
    hipLaunchKernelGGL((k_energy<float>), dim3((unsigned)h->ne), dim3(64), 0, h->stream, h->ne,
                       h->ref.L, h->ref.Q, (const double*)h->Vd.p, (const double*)h->wqd.p,
                       (const float*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                       (const double*)h->geo.p, (const double*)h->mat.p, h->amax, 1e-15, part);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, h->stream, h->ne, part, E);
  HIPCHK(h, hipGetLastError());
  return DGD_OK;
}

dgd_status dgd_wavespeed_change(dgd_handle* h, double* out) {
  if (!h || !out) return DGD_EINVAL;
  if (!h->have_state || !h->have_mat || !h->have_params)
    return fail(h, DGD_ESTATE, "state, material and params needed");
  dgd_status s = dalloc(h, h->tmp, (size_t)h->ne * sizeof(double));
  if (s) return s;
  hipLaunchKernelGGL(k_wavespeed, dim3((unsigned)((h->ne + 255) / 256)), dim3(256), 0, h->stream,
                     h->ne, h->ref.L, (const double*)h->Ua[h->cur].p, (const double*)h->mat.p,
                     h->amax, h->phi0_mean, h->law, (double*)h->tmp.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, h->tmp.p, (size_t)h->ne * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->tmp.release();
  return DGD_OK;
}

dgd_status dgd_set_profiling(dgd_handle* h, int on) {
  if (!h) return DGD_EINVAL;
  h->profiling = on != 0;
  return DGD_OK;
}

dgd_status dgd_get_kernel_times(dgd_handle* h, double* ms, int64_t* launches) {
  if (!h || !ms || !launches) return DGD_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int k = 0; k < DGD_NUM_KERNEL_CLASSES; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& u : h->ev_used) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, u.second.first, u.second.second) == hipSuccess) {
      ms[u.first] += t;
      launches[u.first] += 1;
    }
    h->ev_pool.push_back(u.second.first);
    h->ev_pool.push_back(u.second.second);
  }
  h->ev_used.clear();
  return DGD_OK;
}

dgd_status dgd_get_time_point_states(dgd_handle* h, double* out) {
  if (!h || !out) return DGD_EINVAL;
  if (!h->have_state) return fail(h, DGD_ESTATE, "no state");
  // device layout [e][z][l][10] -> [e][z][p][l]
  const size_t L = h->ref.L, Nt = h->ref.Nt;
  const size_t n = (size_t)h->ne * Nt * L * 10;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<double> tmp(n);
  if (h->prec == DGD_FP64) {
    HIPCHK(h, hipMemcpy(tmp.data(), h->Uz.p, n * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tf(n);
    HIPCHK(h, hipMemcpy(tf.data(), h->Uz.p, n * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) tmp[i] = tf[i];
  }
  for (size_t e = 0; e < (size_t)h->ne; ++e)
    for (size_t z = 0; z < Nt; ++z)
      for (size_t p = 0; p < 10; ++p)
        for (size_t l = 0; l < L; ++l)
          out[((e * Nt + z) * 10 + p) * L + l] = tmp[((e * Nt + z) * L + l) * 10 + p];
  return DGD_OK;
}

dgd_status dgd_adjoint_step(dgd_handle* h, const double* state_n, double* lam,
                            const double* dJ_dseis_n, double* grad_mu0, double* grad_cd) {
  if (!h) return DGD_EINVAL;
  if (!state_n || !lam) return fail(h, DGD_EINVAL, "null state or adjoint state");
  if (h->law != 0) return fail(h, DGD_EINVAL, "the adjoint is that of the continuum-damage law");
  if (h->predictor != 0)
    return fail(h, DGD_EINVAL, "the adjoint is that of the Cauchy-Kovalevskaya predictor");
  if (!h->have_mesh || !h->have_mat || !h->have_params)
    return fail(h, DGD_ESTATE, "mesh, material and params are needed");
  const size_t E = (size_t)h->ne, L = h->ref.L;
  dgd_status s;
  if ((s = alloc_adjoint(h)) || (s = dalloc(h, h->st9, E * 9 * L * h->tsize)) ||
      (s = dalloc(h, h->sta, E * L * sizeof(double))))
    return s;
  const long long n = (long long)(E * 10 * L);
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (h->prec == DGD_FP64) {
    hipLaunchKernelGGL((k_from_f64<double>), g, b, 0, h->stream, h->ne, h->ref.L, state_n,
                       (double*)h->st9.p, (double*)h->sta.p);
    launch_lam_from_f64<double>(h, lam, h->lam[0].p);
  } else {
    hipLaunchKernelGGL((k_from_f64<float>), g, b, 0, h->stream, h->ne, h->ref.L, state_n,
                       (float*)h->st9.p, (double*)h->sta.p);
    launch_lam_from_f64<float>(h, lam, h->lam[0].p);
  }
  if (dJ_dseis_n && h->nrec > 0) {
    if (h->prec == DGD_FP64)
      hipLaunchKernelGGL((k_adj_receivers<double>), dim3(1), dim3(3 * L), 0, h->stream, h->nrec,
                         (int)L, adj_kpl(h), (const long long*)h->r_elem.p, (const double*)h->r_phi.p,
                         dJ_dseis_n, (double*)h->lam[0].p);
    else
      hipLaunchKernelGGL((k_adj_receivers<float>), dim3(1), dim3(3 * L), 0, h->stream, h->nrec,
                         (int)L, adj_kpl(h), (const long long*)h->r_elem.p, (const double*)h->r_phi.p,
                         dJ_dseis_n, (float*)h->lam[0].p);
  }
  HIPCHK(h, hipGetLastError());
  // the caller's gradient arrays take the accumulation directly
  s = dispatch<AdjStepFn>(h, (const void*)h->st9.p, (const double*)h->sta.p,
                          (const void*)h->lam[0].p, h->lam[1].p, (void*)nullptr,
                          (const void*)nullptr, (const void*)nullptr, grad_mu0, grad_cd);
  if (s) return s;
  if (h->prec == DGD_FP64)
    launch_lam_to_f64<double>(h, h->lam[1].p, lam);
  else
    launch_lam_to_f64<float>(h, h->lam[1].p, lam);
  HIPCHK(h, hipGetLastError());
  return DGD_OK;
}

dgd_status dgd_adjoint_step_host(dgd_handle* h, const double* lam_next, double* lam_out,
                                 double* grad_mu0, double* grad_cd) {
  if (!h || !lam_next || !lam_out) return DGD_EINVAL;
  if (h->law != 0) return fail(h, DGD_EINVAL, "the adjoint is that of the continuum-damage law");
  if (h->predictor != 0)
    return fail(h, DGD_EINVAL, "the adjoint is that of the Cauchy-Kovalevskaya predictor");
  if (!h->have_mesh || !h->have_mat || !h->have_params || !h->have_state)
    return fail(h, DGD_ESTATE, "mesh, material, params and state are needed");
  dgd_status s = alloc_adjoint(h);
  if (s) return s;
  const size_t n = (size_t)h->ne * 10 * h->ref.L;
  if ((s = dalloc(h, h->tmp, n * sizeof(double)))) return s;
  HIPCHK(h, hipMemcpyAsync(h->tmp.p, lam_next, n * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
  if (h->prec == DGD_FP64)
    launch_lam_from_f64<double>(h, (const double*)h->tmp.p, h->lam[0].p);
  else
    launch_lam_from_f64<float>(h, (const double*)h->tmp.p, h->lam[0].p);
  HIPCHK(h, hipGetLastError());
  if ((s = dispatch<AdjStepFn>(h, (const void*)h->U9[h->cur].p, (const double*)h->Ua[h->cur].p,
                               (const void*)h->lam[0].p, h->lam[1].p, (void*)nullptr,
                               (const void*)nullptr, (const void*)nullptr, (double*)nullptr,
                               (double*)nullptr)))
    return s;
  if (h->prec == DGD_FP64)
    launch_lam_to_f64<double>(h, h->lam[1].p, (double*)h->tmp.p);
  else
    launch_lam_to_f64<float>(h, h->lam[1].p, (double*)h->tmp.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(lam_out, h->tmp.p, n * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  if (grad_mu0)
    HIPCHK(h, hipMemcpyAsync(grad_mu0, h->gmu.p, (size_t)h->ne * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  if (grad_cd)
    HIPCHK(h, hipMemcpyAsync(grad_cd, h->gcd.p, (size_t)h->ne * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->tmp.release();
  return DGD_OK;
}

dgd_status dgd_forward_checkpointed(dgd_handle* h, int64_t nsteps, int64_t every) {
  if (!h) return DGD_EINVAL;
  if (nsteps < 1 || every < 1) return fail(h, DGD_EINVAL, "nsteps >= 1 and every >= 1 needed");
  if (h->law != 0) return fail(h, DGD_EINVAL, "the adjoint is that of the continuum-damage law");
  if (h->predictor != 0)
    return fail(h, DGD_EINVAL, "the adjoint is that of the Cauchy-Kovalevskaya predictor");
  if (!h->have_mesh || !h->have_mat || !h->have_params || !h->have_state)
    return fail(h, DGD_ESTATE, "mesh, material, params and state are needed before step");
  release_tape(h);
  dgd_status s = ensure_seis(h, nsteps);
  if (s) return s;
  const size_t E = (size_t)h->ne, L = h->ref.L;
  const long long nck = (nsteps + every - 1) / every;
  h->ck9.resize(nck);
  h->cka.resize(nck);
  h->ck_t.resize(nck);
  h->tape_seis0 = h->nrec_steps;
  for (long long c = 0; c < nck; ++c) {
    if ((s = dalloc(h, h->ck9[c], E * 9 * L * h->tsize)) ||
        (s = dalloc(h, h->cka[c], E * L * sizeof(double)))) {
      release_tape(h);
      return s;
    }
    if ((s = copy_state(h, h->ck9[c].p, h->cka[c].p, h->U9[h->cur].p, h->Ua[h->cur].p))) return s;
    h->ck_t[c] = h->t;
    const long long chunk = std::min<long long>(every, nsteps - c * every);
    if ((s = dispatch<StepFn>(h, chunk))) return s;
  }
  if ((s = dgd_synchronize(h))) return s;
  h->tape = true;
  h->tape_id = ++h->tapes_made;
  h->tape_steps = nsteps;
  h->tape_every = every;
  return DGD_OK;
}

dgd_status dgd_backward(dgd_handle* h, const double* dl_dseis, double* grad_mu0, double* grad_cd,
                        double* grad_u0) {
  if (!h) return DGD_EINVAL;
  if (!h->tape) return fail(h, DGD_ESTATE, "no checkpointed forward run to differentiate");
  if (h->nrec > 0 && !dl_dseis) return fail(h, DGD_EINVAL, "null seismogram cotangent");
  if (!grad_mu0 || !grad_cd) return fail(h, DGD_EINVAL, "null gradient output");
  const size_t E = (size_t)h->ne, L = h->ref.L;
  const long long nsteps = h->tape_steps, every = h->tape_every;
  const int nrec = h->nrec;
  for (size_t c = 0; c < h->ck9.size(); ++c)
    if (h->ck9[c].n != E * 9 * L * h->tsize || h->cka[c].n != E * L * sizeof(double))
      return fail(h, DGD_ESTATE, "checkpoints do not match the mesh");
  dgd_status s = alloc_adjoint(h);
  if (s) return s;
  if ((s = dalloc(h, h->save9, E * 9 * L * h->tsize)) ||
      (s = dalloc(h, h->savea, E * L * sizeof(double))) ||
      (s = dalloc(h, h->seg9, (size_t)every * E * 9 * L * h->tsize)) ||
      (s = dalloc(h, h->sega, (size_t)every * E * L * sizeof(double))))
    return s;
  // time-point states of every step of a segment, kept from the replay so
  // that the adjoint need not recompute them (skipped if memory is short,
  // and under a split-BF16 forward, whose predictions are not the FP32
  // adjoint's)
  const size_t uzb = uz_bytes(h);
  bool keep_uz = h->prec != DGD_BF16 && alloc_uz(h, h->seguz, (size_t)every) == DGD_OK;
  if (!keep_uz) {
    (void)hipGetLastError();
    h->err.clear();
  }
  // and the predictor's derivatives and cell-averaged tangents, so that the
  // adjoint need not repeat the prediction either
  const size_t db = E * (size_t)h->N * h->kpl * 16 * h->tsize, ab = E * 48 * h->tsize;
  bool keep_d = keep_uz && dalloc(h, h->segd, (size_t)every * db) == DGD_OK &&
                dalloc(h, h->segacc, (size_t)every * ab) == DGD_OK;
  if (!keep_d) {
    (void)hipGetLastError();
    h->err.clear();
    h->segd.release();
    h->segacc.release();
  }
  if (nrec > 0) {
    if ((s = dalloc(h, h->dlds, (size_t)nsteps * nrec * 3 * sizeof(double)))) return s;
    HIPCHK(h, hipMemcpyAsync(h->dlds.p, dl_dseis, (size_t)nsteps * nrec * 3 * sizeof(double),
                             hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(h, hipMemsetAsync(h->lam[0].p, 0, lam_elems(h) * h->tsize, h->stream));
  if ((s = copy_state(h, h->save9.p, h->savea.p, h->U9[h->cur].p, h->Ua[h->cur].p))) return s;
  const double t_save = h->t;
  const bool prof = h->profiling;
  int lc = 0;
  h->nrec = 0;   // the replay records nothing
  const long long nck = (long long)h->ck9.size();
  for (long long c = nck - 1; c >= 0 && s == DGD_OK; --c) {
    const long long j0 = c * every, j1 = std::min<long long>(j0 + every, nsteps);
    if ((s = copy_state(h, h->U9[h->cur].p, h->Ua[h->cur].p, h->ck9[c].p, h->cka[c].p))) break;
    h->t = h->ck_t[c];
    h->profiling = false;
    for (long long j = j0; j < j1 && s == DGD_OK; ++j) {
      char* d9 = (char*)h->seg9.p + (size_t)(j - j0) * E * 9 * L * h->tsize;
      char* da = (char*)h->sega.p + (size_t)(j - j0) * E * L * sizeof(double);
      if ((s = copy_state(h, d9, da, h->U9[h->cur].p, h->Ua[h->cur].p))) break;
      if (keep_uz) {
        h->uz_override = (char*)h->seguz.p + (size_t)(j - j0) * uzb;
        if (keep_d) {
          h->d_keep = (char*)h->segd.p + (size_t)(j - j0) * db;
          h->acc_keep = (char*)h->segacc.p + (size_t)(j - j0) * ab;
        }
        // the segment's last state is not stepped further: its prediction suffices
        s = (j + 1 < j1) ? dispatch<StepFn>(h, 1) : dispatch<PredictFn>(h);
        h->uz_override = h->d_keep = h->acc_keep = nullptr;
      } else if (j + 1 < j1) {
        s = dispatch<StepFn>(h, 1);
      }
    }
    h->profiling = prof;
    for (long long j = j1 - 1; j >= j0 && s == DGD_OK; --j) {
      if (nrec > 0) {
        const double* g = (const double*)h->dlds.p + (size_t)j * nrec * 3;
        timed(h, 7, [&] {
          if (h->prec == DGD_FP64)
            hipLaunchKernelGGL((k_adj_receivers<double>), dim3(1), dim3(3 * L), 0, h->stream, nrec,
                               (int)L, adj_kpl(h), (const long long*)h->r_elem.p,
                               (const double*)h->r_phi.p, g, (double*)h->lam[lc].p);
          else
            hipLaunchKernelGGL((k_adj_receivers<float>), dim3(1), dim3(3 * L), 0, h->stream, nrec,
                               (int)L, adj_kpl(h), (const long long*)h->r_elem.p,
                               (const double*)h->r_phi.p, g, (float*)h->lam[lc].p);
        });
      }
      const char* u9 = (const char*)h->seg9.p + (size_t)(j - j0) * E * 9 * L * h->tsize;
      const double* ua = (const double*)((const char*)h->sega.p + (size_t)(j - j0) * E * L * sizeof(double));
      void* uz = keep_uz ? (void*)((char*)h->seguz.p + (size_t)(j - j0) * uzb) : nullptr;
      const void* dk = keep_d ? (const void*)((char*)h->segd.p + (size_t)(j - j0) * db) : nullptr;
      const void* ak = keep_d ? (const void*)((char*)h->segacc.p + (size_t)(j - j0) * ab) : nullptr;
      s = dispatch<AdjStepFn>(h, (const void*)u9, ua, (const void*)h->lam[lc].p, h->lam[1 - lc].p,
                              uz, dk, ak, (double*)nullptr, (double*)nullptr);
      lc = 1 - lc;
    }
  }
  h->nrec = nrec;
  h->profiling = prof;
  const dgd_status s2 = copy_state(h, h->U9[h->cur].p, h->Ua[h->cur].p, h->save9.p, h->savea.p);
  h->t = t_save;
  if (s) return s;
  if (s2) return s2;
  HIPCHK(h, hipMemcpyAsync(grad_mu0, h->gmu.p, E * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(grad_cd, h->gcd.p, E * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (grad_u0) {
    const size_t n = E * 10 * L;
    if ((s = dalloc(h, h->tmp, n * sizeof(double)))) return s;
    if (h->prec == DGD_FP64)
      launch_lam_to_f64<double>(h, h->lam[lc].p, (double*)h->tmp.p);
    else
      launch_lam_to_f64<float>(h, h->lam[lc].p, (double*)h->tmp.p);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(grad_u0, h->tmp.p, n * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->tmp.release();
  h->seg9.release();
  h->sega.release();
  h->seguz.release();
  h->segd.release();
  h->segacc.release();
  return DGD_OK;
}

dgd_status dgd_tape_id(const dgd_handle* h, int64_t* id) {
  if (!h || !id) return DGD_EINVAL;
  *id = h->tape_id;
  return DGD_OK;
}

dgd_status dgd_release_tape(dgd_handle* h) {
  if (!h) return DGD_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  release_tape(h);
  return DGD_OK;
}

}  // extern "C"
