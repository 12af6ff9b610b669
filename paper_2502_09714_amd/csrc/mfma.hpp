// Wave-level matrix-core helpers for gfx950 (CDNA4), one 64-lane wavefront.
//
// Every reference-matrix contraction of the step is C(M x 16) += A(M x K) B(K x 16)
// with A a reference matrix (shared by all elements, pre-packed on the host in
// fragment order so that one fragment is one coalesced load) and B a
// per-element matrix with the 10 conservative variables in its 16 columns.
// Fragment layout of the 16x16xK instructions (lane l, 0..63):
//   A: row l%16, k = KS*s + (KS/4)*(l/16) + j      (j < KS/4)
//   B: col l%16, same k
//   C: col l%16, rows 4*(l/16) + i (FP32 accumulators) or (l/16) + 4*i
//      (FP64 accumulators)                                          (i < 4)
// KS = 4 for FP64 / FP32 (v_mfma_*_16x16x4), KS = 16 for BF16 inputs
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// BF16 form: a single BF16 product keeps 8 significant bits of every operand
// (relative rounding 2^-9), which perturbs the discrete operators enough that
// the state drifts from the FP32/FP64 result by more than 3e-3 within tens
// of steps.  Each FP32 operand x is therefore split into x_hi = bf16(x) and
// x_lo = bf16(x - x_hi), and A B is accumulated in FP32 as
// A_lo B_hi + A_hi B_lo + A_hi B_hi (three matrix-core products; the dropped
// A_lo B_lo and the rounding of the low parts are about 2^-17 relative).
// Reference matrices are split on the host, per-element operands when they
// are loaded (v_cvt_pk_bf16_f32, round to nearest even).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Depths of the register rings in the helpers below: how far ahead of its use
// a fragment is requested from L2/HBM (each slot costs one fragment per tile
// row in registers).
//   DGD_PF_STEPS   matrix-core steps, A only: wave_gemm, wave_gemm2, wave_gemm_col9
//   DGD_PF_SHARED  matrix-core steps, A and B: wave_gemm_shared_a
//   DGD_PF_TILES   single products, A only: wave_gemm_tiles
#ifndef DGD_PF_STEPS
#define DGD_PF_STEPS 4
#endif
#ifndef DGD_PF_SHARED
#define DGD_PF_SHARED 2
#endif
#ifndef DGD_PF_TILES
#define DGD_PF_TILES 4
#endif

namespace dgd {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// high and low BF16 parts of four FP32 values (one matrix-core fragment)
struct __attribute__((aligned(16))) bf16s {
  bf16x4 hi, lo;
};

__device__ inline void split_pair(float a, float b, short& ha, short& hb, short& la, short& lb) {
  const __bf16 h0 = (__bf16)a, h1 = (__bf16)b;
  const __bf16 l0 = (__bf16)(a - (float)h0), l1 = (__bf16)(b - (float)h1);
  ha = __builtin_bit_cast(short, h0);
  hb = __builtin_bit_cast(short, h1);
  la = __builtin_bit_cast(short, l0);
  lb = __builtin_bit_cast(short, l1);
}

__device__ inline bf16s split4(float x0, float x1, float x2, float x3) {
  bf16s r;
  short h0, h1, h2, h3, l0, l1, l2, l3;
  split_pair(x0, x1, h0, h1, l0, l1);
  split_pair(x2, x3, h2, h3, l2, l3);
  r.hi = (bf16x4){h0, h1, h2, h3};
  r.lo = (bf16x4){l0, l1, l2, l3};
  return r;
}

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

__host__ __device__ inline uint16_t f32_to_bf16(float x) {
  // round to nearest even (inputs are finite)
  union { float f; uint32_t u; } v;
  v.f = x;
  uint32_t lsb = (v.u >> 16) & 1u;
  v.u += 0x7fffu + lsb;
  return (uint16_t)(v.u >> 16);
}

template <int P> struct Prec;

// Column of a B fragment a lane reads from a [K][RS] matrix that holds NC < 16
// columns: the lanes of the missing columns read column NC, a padding column
// that holds zero in every row.
template <int NC>
__device__ inline int bcol(int lane) {
  const int n = lane & 15;
  return NC < 16 && n > NC ? NC : n;
}

template <> struct Prec<PREC_F64> {
  using T = double;
  using Acc = f64x4;
  using AF = double;
  static constexpr int KS = 4;
  __device__ static inline int crow(int lane, int i) { return (lane >> 4) + 4 * i; }
  __device__ static inline Acc mma(AF a, AF b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // B fragment from a [K][RS] row-major matrix (LDS or global)
  template <int RS, int NC = 16>
  __device__ static inline AF loadB(const T* B, int s, int lane) {
    return B[(KS * s + (lane >> 4)) * RS + bcol<NC>(lane)];
  }
  __device__ static inline AF loadB9(const T* v, int s, int lane) {
    return (lane & 15) == 9 ? v[KS * s + (lane >> 4)] : 0.0;
  }
};

template <> struct Prec<PREC_F32> {
  using T = float;
  using Acc = f32x4;
  using AF = float;
  static constexpr int KS = 4;
  __device__ static inline int crow(int lane, int i) { return 4 * (lane >> 4) + i; }
  __device__ static inline Acc mma(AF a, AF b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  template <int RS, int NC = 16>
  __device__ static inline AF loadB(const T* B, int s, int lane) {
    return B[(KS * s + (lane >> 4)) * RS + bcol<NC>(lane)];
  }
  __device__ static inline AF loadB9(const T* v, int s, int lane) {
    return (lane & 15) == 9 ? v[KS * s + (lane >> 4)] : 0.0f;
  }
};

template <> struct Prec<PREC_BF16> {
  using T = float;
  using Acc = f32x4;
  using AF = bf16s;
  static constexpr int KS = 16;
  __device__ static inline int crow(int lane, int i) { return 4 * (lane >> 4) + i; }
  __device__ static inline Acc mma(const AF& a, const AF& b, Acc c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
  }
  template <int RS, int NC = 16>
  __device__ static inline AF loadB(const T* B, int s, int lane) {
    int k0 = KS * s + 4 * (lane >> 4), n = bcol<NC>(lane);
    return split4(B[(k0 + 0) * RS + n], B[(k0 + 1) * RS + n], B[(k0 + 2) * RS + n],
                  B[(k0 + 3) * RS + n]);
  }
  __device__ static inline AF loadB9(const T* v, int s, int lane) {
    int k0 = KS * s + 4 * (lane >> 4);
    const bool on = (lane & 15) == 9;
    return split4(on ? v[k0] : 0.0f, on ? v[k0 + 1] : 0.0f, on ? v[k0 + 2] : 0.0f,
                  on ? v[k0 + 3] : 0.0f);
  }
};

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Row stride of per-element [rows][16-column] matrices that are read or
// written one row per lane.  A stride of 16 puts those rows on 4 of the 64
// banks; 18 elements (72 B for floats, 8-byte aligned rows; 144 B for
// doubles) spread them over all banks and cost at most two-way conflicts in
// the matrix-core fragment loads and stores.
template <class T> struct Lds { static constexpr int RS = 18; };

// The cell average of the tangent and the damage-source projections keep FP32
// matrix-core inputs in the BF16 form (they feed the FP64 damage update).
template <int P> struct Accurate { static constexpr int value = P == PREC_BF16 ? PREC_F32 : P; };

// C (tiles of 16 rows) += A_packed x B, A packed as [tile][kstep][lane], B a
// [K][RS] row-major matrix (RS = 16 for the global time-point states) whose
// columns from NC on are zero (column NC is stored and zero, see bcol).
// KSTEPS is a compile-time constant so that the loop unrolls and the A-fragment
// loads are issued ahead of the matrix-core instructions that consume them.
// PF false leaves the loads to the compiler's schedule (where B comes from HBM
// as well and two independent products are interleaved by the caller).
template <int P, int MT, int KSTEPS, int RS = Lds<typename Prec<P>::T>::RS, int KSTRIDE = KSTEPS,
          int NC = 16, bool PF = true>
__device__ inline void wave_gemm(const typename Prec<P>::AF* __restrict__ Apk,
                                 const typename Prec<P>::T* B, typename Prec<P>::Acc (&C)[MT],
                                 int lane) {
  using PR = Prec<P>;
  using AF = typename PR::AF;
  if constexpr (!PF) {
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      const AF b = PR::template loadB<RS, NC>(B, s, lane);
#pragma unroll
      for (int t = 0; t < MT; ++t) C[t] = PR::mma(Apk[((size_t)t * KSTRIDE + s) * 64 + lane], b, C[t]);
    }
    return;
  }
  // A fragments of step s + PD requested before the products of step s (see
  // wave_gemm2)
  constexpr int PD = DGD_PF_STEPS, NB = PD + 1;
  AF a[NB][MT];
#pragma unroll
  for (int s = 0; s < PD && s < KSTEPS; ++s)
#pragma unroll
    for (int t = 0; t < MT; ++t) a[s % NB][t] = Apk[((size_t)t * KSTRIDE + s) * 64 + lane];
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    if (s + PD < KSTEPS) {
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[(s + PD) % NB][t] = Apk[((size_t)t * KSTRIDE + s + PD) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    const AF b = PR::template loadB<RS, NC>(B, s, lane);
#pragma unroll
    for (int t = 0; t < MT; ++t) C[t] = PR::mma(a[s % NB][t], b, C[t]);
  }
}

// C[z] += A x B_z for NZ matrices B_z = B + z BSTRIDE ([K][RS] each) that share
// the packed A: every A fragment is loaded once for all of them.
template <int P, int MT, int KSTEPS, int NZ, int RS, int BSTRIDE>
__device__ inline void wave_gemm_shared_a(const typename Prec<P>::AF* __restrict__ Apk,
                                          const typename Prec<P>::T* B,
                                          typename Prec<P>::Acc (&C)[NZ][MT], int lane) {
  using PR = Prec<P>;
  using AF = typename PR::AF;
  // A and B fragments (A from L2/HBM, B from HBM or LDS) PD steps ahead (see
  // wave_gemm2); the NZ x MT products of a step cover their latency
  constexpr int PD = DGD_PF_SHARED, NB = PD + 1;
  AF a[NB][MT], b[NB][NZ];
#pragma unroll
  for (int s = 0; s < PD && s < KSTEPS; ++s) {
#pragma unroll
    for (int t = 0; t < MT; ++t) a[s % NB][t] = Apk[((size_t)t * KSTEPS + s) * 64 + lane];
#pragma unroll
    for (int z = 0; z < NZ; ++z) b[s % NB][z] = PR::template loadB<RS>(B + z * BSTRIDE, s, lane);
  }
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    if (s + PD < KSTEPS) {
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[(s + PD) % NB][t] = Apk[((size_t)t * KSTEPS + s + PD) * 64 + lane];
#pragma unroll
      for (int z = 0; z < NZ; ++z)
        b[(s + PD) % NB][z] = PR::template loadB<RS>(B + z * BSTRIDE, s + PD, lane);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int z = 0; z < NZ; ++z) C[z][t] = PR::mma(a[s % NB][t], b[s % NB][z], C[z][t]);
  }
}

// As wave_gemm, one output tile after the other (each B fragment is read once
// per tile): fewer A fragments in flight, for kernels short of registers.
template <int P, int MT, int KSTEPS, int RS = Lds<typename Prec<P>::T>::RS>
__device__ inline void wave_gemm_tiles(const typename Prec<P>::AF* __restrict__ Apk,
                                       const typename Prec<P>::T* B,
                                       typename Prec<P>::Acc (&C)[MT], int lane) {
  using PR = Prec<P>;
  using AF = typename PR::AF;
  // A fragments PD products ahead, in the order they are used (see wave_gemm2)
  constexpr int NS = MT * KSTEPS, PD = DGD_PF_TILES, NB = PD + 1;
  AF a[NB];
#pragma unroll
  for (int k = 0; k < PD && k < NS; ++k) a[k % NB] = Apk[(size_t)k * 64 + lane];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k + PD < NS) a[(k + PD) % NB] = Apk[(size_t)(k + PD) * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    const int t = k / KSTEPS, s = k % KSTEPS;
    C[t] = PR::mma(a[k % NB], PR::template loadB<RS>(B, s, lane), C[t]);
  }
}

// C += A x B for a B of 32 columns (two 16-column tiles, row stride RS): each
// A fragment feeds two matrix-core products.
template <int P, int MT, int KSTEPS, int RS>
__device__ inline void wave_gemm2(const typename Prec<P>::AF* __restrict__ Apk,
                                  const typename Prec<P>::T* B, typename Prec<P>::Acc (&C)[MT][2],
                                  int lane) {
  using PR = Prec<P>;
  using AF = typename PR::AF;
  // A fragments come from L2/HBM: those of step s + PD are requested before
  // the products of step s are issued (the scheduling fence keeps the
  // compiler from sinking the loads down to their use), so that PD steps of
  // matrix-core work cover their latency
  constexpr int PD = DGD_PF_STEPS, NB = PD + 1;
  AF a[NB][MT];
#pragma unroll
  for (int s = 0; s < PD && s < KSTEPS; ++s)
#pragma unroll
    for (int t = 0; t < MT; ++t) a[s % NB][t] = Apk[((size_t)t * KSTEPS + s) * 64 + lane];
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    if (s + PD < KSTEPS) {
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[(s + PD) % NB][t] = Apk[((size_t)t * KSTEPS + s + PD) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    const AF b0 = PR::template loadB<RS>(B, s, lane);
    const AF b1 = PR::template loadB<RS>(B + 16, s, lane);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      C[t][0] = PR::mma(a[s % NB][t], b0, C[t][0]);
      C[t][1] = PR::mma(a[s % NB][t], b1, C[t][1]);
    }
  }
}

template <int P, int MT>
__device__ inline void zero_C2(typename Prec<P>::Acc (&C)[MT][2]) {
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) C[t][h][i] = 0;
}

// Store 32-column C tiles to a [rows][RS] matrix, rows >= rmax dropped, times scale.
template <int P, int MT, int RS>
__device__ inline void store_C2(const typename Prec<P>::Acc (&C)[MT][2], typename Prec<P>::T* dst,
                                int rmax, typename Prec<P>::T scale, int lane) {
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * t + Prec<P>::crow(lane, i);
        if (r < rmax) dst[r * RS + 16 * h + (lane & 15)] = scale * C[t][h][i];
      }
}

// C += A x B with B[k][n] = (n == 9) ? v[k] : 0 (a vector placed in the damage column)
template <int P, int MT, int KSTEPS>
__device__ inline void wave_gemm_col9(const typename Prec<P>::AF* __restrict__ Apk,
                                      const typename Prec<P>::T* v, typename Prec<P>::Acc (&C)[MT],
                                      int lane) {
  using PR = Prec<P>;
  using AF = typename PR::AF;
  // A fragments of step s + PD requested before the products of step s (see
  // wave_gemm2)
  constexpr int PD = DGD_PF_STEPS, NB = PD + 1;
  AF a[NB][MT];
#pragma unroll
  for (int s = 0; s < PD && s < KSTEPS; ++s)
#pragma unroll
    for (int t = 0; t < MT; ++t) a[s % NB][t] = Apk[((size_t)t * KSTEPS + s) * 64 + lane];
#pragma unroll
  for (int s = 0; s < KSTEPS; ++s) {
    if (s + PD < KSTEPS) {
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[(s + PD) % NB][t] = Apk[((size_t)t * KSTEPS + s + PD) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    const AF b = PR::loadB9(v, s, lane);
#pragma unroll
    for (int t = 0; t < MT; ++t) C[t] = PR::mma(a[s % NB][t], b, C[t]);
  }
}

// Store C tiles to a [rows][RS] matrix, rows >= rmax and columns >= CMAX
// dropped, times scale.
template <int P, int MT, int RS = Lds<typename Prec<P>::T>::RS, int CMAX = 16>
__device__ inline void store_C(const typename Prec<P>::Acc (&C)[MT], typename Prec<P>::T* dst,
                               int rmax, typename Prec<P>::T scale, int lane) {
  static_assert(CMAX <= RS, "stored columns fit the row stride");
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = 16 * t + Prec<P>::crow(lane, i);
      if (r < rmax && (CMAX == 16 || (lane & 15) < CMAX)) dst[r * RS + (lane & 15)] = scale * C[t][i];
    }
}

template <int P, int MT>
__device__ inline void zero_C(typename Prec<P>::Acc (&C)[MT]) {
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) C[t][i] = 0;
}

}  // namespace dgd
