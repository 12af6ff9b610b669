// Pointwise derivatives for the discrete adjoint of the CDM step (device).
//
// Vector-Jacobian products of every pointwise map of the forward step, with
// respect to the state u (10 quantities) and the shear modulus mu0 (and C_d
// where it enters).  Conventions shared with the forward kernels:
//   * alpha clamp: derivative 1 on the closed interval [0, alpha_max], else 0;
//   * damage-rate threshold xi > xi0 and the sqrt(I2) guard: derivative 0 on
//     the inactive side;
//   * LLF constant C = max(c-, c+): at an exact tie each side takes one half.
// Flux and stress products are exact through the hand-written tangent; the
// derivatives of the tangent itself (predictor) and of the boundary fluxes use
// forward-mode dual numbers; the derivative of the largest acoustic-tensor
// eigenvalue uses its eigenvector (v^T dQ v), which stays well defined when
// the two smaller eigenvalues coincide.
#pragma once
#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace dgd {

// the overloads for Dual below must not hide the scalar ones
using ::fabs;
using ::fmax;
using ::sqrt;

template <class T> struct Dual {
  T v, d;
  __device__ Dual() : v(0), d(0) {}
  __device__ Dual(T a, T b) : v(a), d(b) {}
  __device__ Dual(double a) : v(T(a)), d(T(0)) {}
  __device__ Dual(float a) : v(T(a)), d(T(0)) {}
  __device__ Dual(int a) : v(T(a)), d(T(0)) {}
};

template <class T> __device__ inline Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> __device__ inline Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> __device__ inline Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> __device__ inline Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> __device__ inline Dual<T> operator/(Dual<T> a, Dual<T> b) {
  const T iv = T(1) / b.v;
  return {a.v * iv, (a.d - a.v * iv * b.d) * iv};
}
template <class T> __device__ inline Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a = a + b; return a; }
template <class T> __device__ inline Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a = a - b; return a; }
template <class T> __device__ inline Dual<T>& operator*=(Dual<T>& a, Dual<T> b) { a = a * b; return a; }
template <class T> __device__ inline bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <class T> __device__ inline bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <class T> __device__ inline bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <class T> __device__ inline bool operator>=(Dual<T> a, Dual<T> b) { return a.v >= b.v; }
template <class T> __device__ inline Dual<T> sqrt(Dual<T> a) {
  const T s = ::sqrt(a.v);
  return {s, s > T(0) ? a.d / (T(2) * s) : T(0)};
}
template <class T> __device__ inline Dual<T> fabs(Dual<T> a) { return a.v < T(0) ? -a : a; }
template <class T> __device__ inline Dual<T> fmax(Dual<T> a, Dual<T> b) { return a.v >= b.v ? a : b; }

template <class T>
__device__ inline MatP<Dual<T>> dual_mat(const MatP<T>& m, bool seed_mu) {
  MatP<Dual<T>> r;
  r.rho = Dual<T>(m.rho, T(0));
  r.lam = Dual<T>(m.lam, T(0));
  r.mu = Dual<T>(m.mu, seed_mu ? T(1) : T(0));
  r.gr = Dual<T>(m.gr, T(0));
  r.xi0 = Dual<T>(m.xi0, T(0));
  r.cd = Dual<T>(m.cd, T(0));
  return r;
}

template <class T>
__device__ inline Law<Dual<T>> dual_law(const Law<T>& l) {
  return Law<Dual<T>>{Dual<T>(l.amax, T(0)), Dual<T>(l.smin, T(0))};
}

// seed direction j (0..9) of the state; j = 10 seeds nothing (material pass)
template <class T>
__device__ inline void dual_state(const T* u, int j, Dual<T>* ud) {
#pragma unroll
  for (int k = 0; k < 10; ++k) ud[k] = Dual<T>(u[k], k == j ? T(1) : T(0));
}

// stress cotangent ls (6) -> state and mu0 cotangents: ls^T d sigma/du in
// closed form.  With sigma_k = coef u_k + e_k iso (e_k = 1 on the normal
// entries), G_q = ds/du_q and Xi_q = dxi/du_q:
//   sum_k ls_k dsigma_k/du_q = coef ls_q + e_q lambda0 tr(ls) - a gamma_r tr(ls) G_q
//                              - a gamma_r (ls . eps) Xi_q,
//   sum_k ls_k dsigma_k/dalpha = clamp' (-gamma_r s tr(ls) + (2 xi0 - xi) gamma_r (ls . eps)),
//   sum_k ls_k dsigma_k/dmu0 = 2 (ls . eps).
template <class T>
__device__ inline void stress_vjp_p(const Parts<T>& p, const T* u, const MatP<T>& m,
                                    const T ls[6], T gu[10], T& gmu) {
  const T agr = p.ac * m.gr;
  const T coef = T(2) * (m.mu + p.ac * m.xi0 * m.gr) - agr * p.xi;
  const T trl = ls[0] + ls[1] + ls[2];
  T lu = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) lu += ls[k] * u[k];
  const T a6 = T(2) * m.xi0 * m.gr;
  if (p.guard) {
#pragma unroll
    for (int q = 0; q < 6; ++q) gu[q] += coef * ls[q] + (q < 3 ? m.lam * trl : T(0));
    gu[9] += p.dac * a6 * lu;
  } else {
    const T im = p.im, is = T(1) / p.sp, is3 = is * is * is;
    T lep = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) lep += ls[k] * u[k] * im;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const T w = q < 3 ? T(1) : T(2);
      const T epq = u[q] * im;
      const T G = w * epq * is;
      const T Xp = (q < 3 ? is : T(0)) - p.I1p * w * epq * is3;
      gu[q] += coef * ls[q] + (q < 3 ? m.lam * trl : T(0)) - agr * (trl * G + lep * Xp);
    }
    gu[9] += p.dac * (-m.gr * p.s * trl + (a6 - m.gr * p.xi) * lu);
  }
  gmu += T(2) * lu;
}

template <class T>
__device__ inline void stress_vjp(const T* u, const MatP<T>& m, const Law<T>& law, const T ls[6],
                                  T gu[10], T& gmu) {
  stress_vjp_p(cdm_parts(u, law), u, m, ls, gu, gmu);
}

// w^T d(F_n)/du for the normal flux F_n = n_d F^d(u)
template <class T>
__device__ inline void normal_flux_vjp(const T* u, const T n[3], const MatP<T>& m,
                                       const Law<T>& law, const T w[10], T gu[10], T& gmu) {
  gu[6] += -w[0] * n[0] - T(0.5) * w[3] * n[1] - T(0.5) * w[5] * n[2];
  gu[7] += -w[1] * n[1] - T(0.5) * w[3] * n[0] - T(0.5) * w[4] * n[2];
  gu[8] += -w[2] * n[2] - T(0.5) * w[4] * n[1] - T(0.5) * w[5] * n[0];
  const T ir = T(1) / m.rho;
  T ls[6];
  ls[0] = -ir * n[0] * w[6];
  ls[1] = -ir * n[1] * w[7];
  ls[2] = -ir * n[2] * w[8];
  ls[3] = -ir * (n[1] * w[6] + n[0] * w[7]);   // sigma_xy appears in rows x (n_y) and y (n_x)
  ls[4] = -ir * (n[2] * w[7] + n[1] * w[8]);
  ls[5] = -ir * (n[0] * w[8] + n[2] * w[6]);
  stress_vjp(u, m, law, ls, gu, gmu);
}

// c = sqrt(lambda_max(rho Q)/rho) and its derivatives with respect to the
// state (10) and mu0.  With v the unit eigenvector of lambda_max, d lambda =
// v^T d(rho Q) v, and
//   v^T (rho Q) v = lambda0 (v.n)^2 + h (1 + (v.n)^2) - 2 c1 (v.n) E + c2 E^2,
//   E = v.(eps n),  h = mu' - a gamma_r xi / 2,  c1 = a gamma_r / s,
//   c2 = a gamma_r I1 / s^3,
// differentiated in closed form (the strain terms in scale-free variables;
// their common factor 1/max|eps| is applied last).
template <class T>
__device__ inline T llf_speed_grad(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law,
                                   T dc[10], T& dcmu) {
  T Q[3][3];
  acoustic_rhoQ(u, n, m, law, Q);
  const T lam = sym3_lmax(Q[0][0], Q[1][1], Q[2][2], Q[0][1], Q[0][2], Q[1][2]);
#pragma unroll
  for (int k = 0; k < 10; ++k) dc[k] = T(0);
  dcmu = T(0);
  const T lm = lam / m.rho;
  if (!(lm > T(0))) return T(0);
  const T c = sqrt(lm);
  // eigenvector of lambda_max: largest cross product of two rows of
  // (Q - lambda I)/lambda (scaled to O(1): squared cross products of the
  // unscaled rows, ~ Q^4 ~ 1e44, overflow FP32)
  const T il = T(1) / lam;
  const T r[3][3] = {{(Q[0][0] - lam) * il, Q[0][1] * il, Q[0][2] * il},
                     {Q[1][0] * il, (Q[1][1] - lam) * il, Q[1][2] * il},
                     {Q[2][0] * il, Q[2][1] * il, (Q[2][2] - lam) * il}};
  T v[3] = {T(0), T(0), T(0)};
  T best = T(-1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3;
    const T x = r[a][1] * r[b][2] - r[a][2] * r[b][1];
    const T y = r[a][2] * r[b][0] - r[a][0] * r[b][2];
    const T z = r[a][0] * r[b][1] - r[a][1] * r[b][0];
    const T nn = x * x + y * y + z * z;
    if (nn > best) {
      best = nn;
      v[0] = x;
      v[1] = y;
      v[2] = z;
    }
  }
  if (!(best > T(0))) return c;
  const T iv = T(1) / sqrt(best);
  v[0] *= iv;
  v[1] *= iv;
  v[2] *= iv;
  const T f = T(1) / (T(2) * c * m.rho);      // dc = d lambda / (2 c rho)
  const Parts<T> p = cdm_parts(u, law);
  const T vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  const T q1 = T(1) + vn * vn;
  dcmu = q1 * f;
  if (p.guard) {
    dc[9] = p.dac * m.xi0 * m.gr * q1 * f;
    return c;
  }
  const T im = p.im, sp = p.sp, I1p = p.I1p;
  const T is = T(1) / sp, is2 = is * is, is3 = is2 * is;
  T ep[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) ep[k] = u[k] * im;
  // E / max|eps| and its derivatives D_j = v.(d eps/du_j n)
  const T en0 = ep[0] * n[0] + ep[3] * n[1] + ep[5] * n[2];
  const T en1 = ep[3] * n[0] + ep[1] * n[1] + ep[4] * n[2];
  const T en2 = ep[5] * n[0] + ep[4] * n[1] + ep[2] * n[2];
  const T ve = v[0] * en0 + v[1] * en1 + v[2] * en2;
  const T D[6] = {v[0] * n[0], v[1] * n[1], v[2] * n[2], v[0] * n[1] + v[1] * n[0],
                  v[1] * n[2] + v[2] * n[1], v[2] * n[0] + v[0] * n[2]};
  const T agr = p.ac * m.gr;
  const T sc = agr * im * f;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T wj = j < 3 ? T(1) : T(2);
    const T ej = j < 3 ? T(1) : T(0);
    const T G = wj * ep[j] * is;                        // ds/du_j
    const T Xi = ej * is - I1p * wj * ep[j] * is3;      // dxi/du_j times max|eps|
    const T t = T(-0.5) * Xi * q1 - T(2) * vn * (D[j] * is - G * ve * is2) +
                ej * ve * ve * is3 - T(3) * I1p * G * ve * ve * is3 * is +
                T(2) * I1p * ve * D[j] * is3;
    dc[j] = sc * t;
  }
  dc[9] = p.dac * f *
          ((m.xi0 * m.gr - T(0.5) * m.gr * p.xi) * q1 - T(2) * m.gr * is * vn * ve +
           m.gr * I1p * is3 * ve * ve);
  return c;
}

// LLF flux F* = (F_n(u-) + F_n(u+))/2 + C (u- - u+)/2: cotangents of u- and of
// the minus-side mu0 for the flux cotangent w
template <class T>
__device__ inline void llf_vjp_minus(const T* um, const T* up, const T n[3], const MatP<T>& mm,
                                     const MatP<T>& mp, const Law<T>& law, const T w[10],
                                     T gu[10], T& gmu) {
  T wh[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) wh[k] = T(0.5) * w[k];
  normal_flux_vjp(um, n, mm, law, wh, gu, gmu);
  T ub[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) ub[k] = T(0.5) * (um[k] + up[k]);
  T d1[10], m1;
  const T c1 = llf_speed_grad(ub, n, mm, law, d1, m1);
  T C = c1, a1 = T(0.5);
  if (!same_material(mm, mp)) {
    T d2[10], m2;
    const T c2 = llf_speed_grad(ub, n, mp, law, d2, m2);
    // tie rule: each side takes one half
    a1 = c1 > c2 ? T(1) : (c1 < c2 ? T(0) : T(0.5));
    const T a2 = T(1) - a1;
    C = c1 > c2 ? c1 : c2;
#pragma unroll
    for (int k = 0; k < 10; ++k) d1[k] = a1 * d1[k] + a2 * d2[k];
  }
  // equal materials: c1 = c2, a tie, and a1 d1 + a2 d2 = d1
  T jump = T(0);
#pragma unroll
  for (int k = 0; k < 10; ++k) jump += w[k] * (um[k] - up[k]);
  // d/du-: C w/2 + (w . jump)/2 * dC/dubar * 1/2
#pragma unroll
  for (int k = 0; k < 10; ++k) gu[k] += T(0.5) * C * w[k] + T(0.25) * jump * d1[k];
  gmu += T(0.5) * jump * a1 * m1;
}

// Both sides at once: cotangents of u- and u+ and of each side's mu0 for the
// flux cotangent w (the flux taken with the normal n of the minus side).
// d/du+ differs from d/du- only in the sign of the C w / 2 term.
template <class T>
__device__ inline void llf_vjp_both(const T* um, const T* up, const T n[3], const MatP<T>& mm,
                                    const MatP<T>& mp, const Law<T>& law, const T w[10],
                                    T gm[10], T gp[10], T& gmum, T& gmup) {
  T wh[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) wh[k] = T(0.5) * w[k];
  normal_flux_vjp(um, n, mm, law, wh, gm, gmum);
  normal_flux_vjp(up, n, mp, law, wh, gp, gmup);
  T ub[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) ub[k] = T(0.5) * (um[k] + up[k]);
  T d1[10], m1, m2;
  const T c1 = llf_speed_grad(ub, n, mm, law, d1, m1);
  T C = c1, a1 = T(0.5);
  m2 = m1;
  if (!same_material(mm, mp)) {
    T d2[10];
    const T c2 = llf_speed_grad(ub, n, mp, law, d2, m2);
    a1 = c1 > c2 ? T(1) : (c1 < c2 ? T(0) : T(0.5));
    const T a2 = T(1) - a1;
    C = c1 > c2 ? c1 : c2;
#pragma unroll
    for (int k = 0; k < 10; ++k) d1[k] = a1 * d1[k] + a2 * d2[k];
  }
  T jump = T(0);
#pragma unroll
  for (int k = 0; k < 10; ++k) jump += w[k] * (um[k] - up[k]);
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const T cw = T(0.5) * C * w[k], dj = T(0.25) * jump * d1[k];
    gm[k] += cw + dj;
    gp[k] += dj - cw;
  }
  gmum += T(0.5) * jump * a1 * m1;
  gmup += T(0.5) * jump * (T(1) - a1) * m2;
}

// boundary flux cotangents by forward-mode dual numbers
template <class T>
__device__ inline void boundary_vjp(int kind, const T* u, const T n[3], const MatP<T>& m,
                                    const Law<T>& law, const T w[10], T gu[10], T& gmu) {
  const Law<Dual<T>> ld = dual_law(law);
  const MatP<Dual<T>> md0 = dual_mat(m, false);
  Dual<T> nd[3] = {Dual<T>(n[0], T(0)), Dual<T>(n[1], T(0)), Dual<T>(n[2], T(0))};
  Dual<T> ud[10], F[10];
  // j = 0..9 seeds one state entry (alpha enters through the clamped moduli);
  // j = 10 seeds mu0
  for (int j = 0; j < 11; ++j) {
    dual_state(u, j, ud);
    const MatP<Dual<T>> md = j == 10 ? dual_mat(m, true) : md0;
    boundary_flux(kind, ud, nd, md, ld, F);
    T s = T(0);
#pragma unroll
    for (int k = 0; k < 10; ++k) s += w[k] * F[k].d;
    if (j == 10)
      gmu += s;
    else
      gu[j] += s;
  }
}

// damage rate r = C_d gamma_r I2 (xi - xi0): state and C_d cotangents for the
// rate cotangent lr
template <class T>
__device__ inline void rate_vjp_p(const Parts<T>& p, const T* u, const MatP<T>& m, T lr, T gu[10],
                                  T& gcd) {
  if (p.guard || !(p.xi > m.xi0)) return;
  // r = C_d gamma_r (I1 s - xi0 I2),  ds/du_q = w_q u_q / s,  I1 / s = xi
  const T k = lr * m.cd * m.gr;
  const T c = p.xi - T(2) * m.xi0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const T wq = q < 3 ? T(1) : T(2);
    gu[q] += k * ((q < 3 ? p.s : T(0)) + c * wq * u[q]);
  }
  gcd += lr * m.gr * p.I2 * (p.xi - m.xi0);
}

template <class T>
__device__ inline void rate_vjp(const T* u, const MatP<T>& m, const Law<T>& law, T lr, T gu[10],
                                T& gcd) {
  rate_vjp_p(cdm_parts(u, law), u, m, lr, gu, gcd);
}

// tangent cotangent lt (6 x 7, the cell-average weight folded in): state
// cotangent through the second derivatives of the stress,
//   gu_j = d/du_j sum_{k,c} lt[k][c] ds[k][c](u),
// in closed form.  With G_q = ds/du_q = w_q u_q / s and Xi_q = dxi/du_q, every
// singular term comes from the I1 sqrt(I2) part of the strain energy; in the
// scale-free variables (eps / max|eps|) the strain derivatives carry one
// factor 1/max|eps|.
template <class T>
__device__ inline void tangent_vjp_p(const Parts<T>& p, const T* u, const MatP<T>& m,
                                     const T lt[6][7], T gu[10]) {
  T trT = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) trT += lt[k][k];
  const T a6 = T(2) * m.xi0 * m.gr;
  if (p.guard) {
    // tangent: delta coef + e e lambda0, alpha column 2 xi0 gamma_r u_k (times dac)
#pragma unroll
    for (int j = 0; j < 6; ++j) gu[j] += p.dac * a6 * lt[j][6];
    gu[9] += p.dac * a6 * trT;
    return;
  }
  const T im = p.im, sp = p.sp, I1p = p.I1p;
  const T is = T(1) / sp, is2 = is * is, is3 = is2 * is;
  T ep[6], G[6], Xp[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T w = k < 3 ? T(1) : T(2);
    ep[k] = u[k] * im;
    G[k] = w * ep[k] * is;
    Xp[k] = (k < 3 ? is : T(0)) - I1p * w * ep[k] * is3;
  }
  // r_q = sum_{k<3} lt[k][q];  a_q = sum_k lt[k][q] ep_k;  (lt Xi)_k
  T r[7], a[6], tX[6];
#pragma unroll
  for (int q = 0; q < 7; ++q) r[q] = lt[0][q] + lt[1][q] + lt[2][q];
  T rG = T(0), aG = T(0), ae = T(0), aX = T(0), t6e = T(0);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) s += lt[k][q] * ep[k];
    a[q] = s;
    rG += r[q] * G[q];
    aG += s * G[q];
    aX += s * Xp[q];
    if (q < 3) ae += s;
    t6e += lt[q][6] * ep[q];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T s = T(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) s += lt[k][q] * Xp[q];
    tX[k] = s;
  }
  const T agr = p.ac * m.gr;
  const T sc = agr * im;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const T wj = j < 3 ? T(1) : T(2);
    const T ej = j < 3 ? T(1) : T(0);
    // d/du_j of the 6 x 6 block: coef, e_k G_q, u_k Xi_q terms
    const T A1 = -Xp[j] * trT;
    const T A2 = -is * (r[j] * wj - G[j] * rG);
    const T A3 = -tX[j];
    const T A4 = (G[j] * ae + ej * aG) * is2 + I1p * wj * a[j] * is3 -
                 T(3) * I1p * G[j] * aG * is3;
    T g = sc * (A1 + A2 + A3 + A4);
    // alpha column: dac (-e_k gamma_r s + (2 xi0 - xi) gamma_r u_k)
    g += p.dac * (-m.gr * G[j] * r[6] - m.gr * Xp[j] * t6e + (a6 - m.gr * p.xi) * lt[j][6]);
    gu[j] += g;
  }
  gu[9] += p.dac * ((a6 - m.gr * p.xi) * trT - m.gr * rG - m.gr * aX);
}

}  // namespace dgd
