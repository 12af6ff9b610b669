// Pointwise continuum-damage (CDM) law, fluxes and boundary fluxes (device).
//
// u = (eps_xx, eps_yy, eps_zz, eps_xy, eps_yz, eps_zx, v_x, v_y, v_z, alpha),
// tensor shear strains.  Stress and damage rate of Eq. cdb-model:
//   sigma = lambda0 I1 delta - a gamma_r sqrt(I2) delta + [2(mu0 + a xi0 gamma_r) - a gamma_r xi] eps
//   r     = C_d gamma_r I2 (xi - xi0) if xi > xi0 else 0,   xi = I1/sqrt(I2)
// with a = clamp(alpha, 0, alpha_max); for sqrt(I2) <= 1e-15 (I2 <= 1e-30) the
// sqrt(I2) and xi terms are dropped and r = 0.  Flux of Eq. nonlinear hyper pdes:
//   F^d(eps_ij) = -(v_i n_j + v_j n_i)/2 (d-component), F^d(v_i) = -sigma_id/rho, F(alpha) = 0.
// The local Lax-Friedrichs constant (Eq. rusanov-flux) is the spectral radius of
// n_d dF^d/du, i.e. sqrt(lambda_max) of the acoustic tensor
//   rho Q = lambda0 n n + (mu' - a gamma_r xi / 2)(I + n n)
//           - (a gamma_r / s)(n (eps n) + (eps n) n) + (a gamma_r I1 / s^3)(eps n)(eps n),
// mu' = mu0 + a xi0 gamma_r, s = sqrt(I2); lambda_max by the trigonometric
// closed form for symmetric 3x3 matrices.
// Boundary fluxes (Appendix A.3) use the isotropic effective moduli
//   lambda_eff = lambda0 - a gamma_r xi / 3,  mu_eff = mu0 + a xi0 gamma_r - a gamma_r xi / 2
// and the closed forms of T B^{1,eff} u^b (free surface: traction-free
// Riemann state) and T R Lambda^+ R^{-1} T^{-1} u (absorbing).
// The internal-variable law of Eq. ivm-model (IvmLaw below) replaces stress,
// rate, tangent, Lax-Friedrichs speed and boundary moduli where a kernel is
// instantiated with it; fluxes and boundary closed forms are shared.
#pragma once
#include <hip/hip_runtime.h>

namespace dgd {

template <class T> struct MatP { T rho, lam, mu, gr, xi0, cd; };

template <class T> struct Law {
  T amax;   // clamp of alpha
  T smin;   // sqrt(I2) at or below which the xi and sqrt(I2) terms are dropped
};

// The rheology of a kernel instantiation: the continuum-damage law (Eq.
// cdb-model) or the internal-variable law (Eq. ivm-model); both defined below.
struct CdmLaw;
struct IvmLaw;

// Invariants computed from the strain scaled by its largest entry, so that the
// scale-free quantities (xi and the tangent / acoustic-tensor directions) are
// the same in FP32 and FP64 down to the guard sqrt(I2) <= smin.
template <class T> struct Parts {
  T I1, I2, s, xi, ac, dac;
  T im;            // 1 / max|eps_k| (0 in the guard)
  T sp, I1p;       // sqrt(I2) and I1 of the scaled strain
  bool guard;
};

template <class T>
__device__ inline Parts<T> cdm_parts(const T* u, const Law<T>& law) {
  Parts<T> p;
  T m = fabs(u[0]);
#pragma unroll
  for (int k = 1; k < 6; ++k) m = fmax(m, fabs(u[k]));
  p.I1 = u[0] + u[1] + u[2];
  // 1 / max|eps| only where it is finite: for max|eps| <= smin/4 (which in
  // FP32 includes denormal strains, whose reciprocal overflows) sqrt(I2) <=
  // 3 max|eps| is inside the guard anyway
  const T im = m > law.smin * T(0.25) ? T(1) / m : T(0);
  const T e0 = u[0] * im, e1 = u[1] * im, e2 = u[2] * im, e3 = u[3] * im, e4 = u[4] * im,
          e5 = u[5] * im;
  const T I2p = e0 * e0 + e1 * e1 + e2 * e2 + T(2) * (e3 * e3 + e4 * e4 + e5 * e5);
  const T sp = sqrt(I2p);
  const T I1p = e0 + e1 + e2;
  const T s = m * sp;
  p.guard = !(s > law.smin);
  p.s = p.guard ? T(0) : s;
  p.I2 = s * s;
  p.sp = p.guard ? T(0) : sp;
  p.I1p = p.guard ? T(0) : I1p;
  p.xi = p.guard ? T(0) : I1p / sp;
  p.im = p.guard ? T(0) : im;
  T a = u[9];
  p.ac = a < T(0) ? T(0) : (a > law.amax ? law.amax : a);
  p.dac = (a >= T(0) && a <= law.amax) ? T(1) : T(0);
  return p;
}

template <class T>
__device__ inline void cdm_stress(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
  Parts<T> p = cdm_parts(u, law);
  T iso = m.lam * p.I1 - p.ac * m.gr * p.s;
  T coef = T(2) * (m.mu + p.ac * m.xi0 * m.gr) - p.ac * m.gr * p.xi;
#pragma unroll
  for (int k = 0; k < 6; ++k) sig[k] = coef * u[k] + (k < 3 ? iso : T(0));
}

// stress and damage rate from one evaluation of the invariants
template <class T>
__device__ inline T cdm_stress_rate(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
  Parts<T> p = cdm_parts(u, law);
  T iso = m.lam * p.I1 - p.ac * m.gr * p.s;
  T coef = T(2) * (m.mu + p.ac * m.xi0 * m.gr) - p.ac * m.gr * p.xi;
#pragma unroll
  for (int k = 0; k < 6; ++k) sig[k] = coef * u[k] + (k < 3 ? iso : T(0));
  if (p.guard || !(p.xi > m.xi0)) return T(0);
  return m.cd * m.gr * p.I2 * (p.xi - m.xi0);
}

template <class T>
__device__ inline T cdm_rate(const T* u, const MatP<T>& m, const Law<T>& law) {
  Parts<T> p = cdm_parts(u, law);
  if (p.guard || !(p.xi > m.xi0)) return T(0);
  return m.cd * m.gr * p.I2 * (p.xi - m.xi0);
}

// d sigma_k / d u_q for q = 0..5 (strain entries, a shear entry standing for
// both eps_ij and eps_ji) and q = 6 (alpha).
template <class T>
__device__ inline void cdm_tangent(const T* u, const MatP<T>& m, const Law<T>& law, T ds[6][7]) {
  Parts<T> p = cdm_parts(u, law);
  const T agr = p.ac * m.gr;
  const T coef = T(2) * (m.mu + p.ac * m.xi0 * m.gr) - agr * p.xi;
  // the 1/sqrt(I2) terms are homogeneous of degree 0: use the scaled strain
  const T is = p.guard ? T(0) : T(1) / p.sp;
  const T is3 = is * is * is;
  T ep[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) ep[k] = u[k] * p.im;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const T w = q < 3 ? T(1) : T(2);
      T v = (k == q) ? coef : T(0);
      if (k < 3 && q < 3) v += m.lam;
      if (k < 3) v -= agr * w * ep[q] * is;
      v -= agr * ep[k] * ((q < 3 ? is : T(0)) - p.I1p * w * ep[q] * is3);
      ds[k][q] = v;
    }
    ds[k][6] = p.dac * ((k < 3 ? -m.gr * p.s : T(0)) + (T(2) * m.xi0 * m.gr - m.gr * p.xi) * u[k]);
  }
}

// index of the symmetric component (i, j) in the six-entry ordering
__device__ __host__ constexpr int sym_idx(int i, int j) {
  return (i == j) ? i : ((i + j == 1) ? 3 : ((i + j == 3) ? 4 : 5));
}

// F_n = n_d F^d(u) for the 10 quantities
template <class LW = CdmLaw, class T>
__device__ inline void normal_flux(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law,
                                   T F[10]) {
  T sig[6];
  LW::stress(u, m, law, sig);
  const T* v = u + 6;
  F[0] = -v[0] * n[0];
  F[1] = -v[1] * n[1];
  F[2] = -v[2] * n[2];
  F[3] = T(-0.5) * (v[0] * n[1] + v[1] * n[0]);
  F[4] = T(-0.5) * (v[1] * n[2] + v[2] * n[1]);
  F[5] = T(-0.5) * (v[2] * n[0] + v[0] * n[2]);
  const T ir = T(1) / m.rho;
  F[6] = -ir * (sig[0] * n[0] + sig[3] * n[1] + sig[5] * n[2]);
  F[7] = -ir * (sig[3] * n[0] + sig[1] * n[1] + sig[4] * n[2]);
  F[8] = -ir * (sig[5] * n[0] + sig[4] * n[1] + sig[2] * n[2]);
  F[9] = T(0);
}

// largest eigenvalue of a symmetric 3x3 matrix (trigonometric closed form)
template <class T>
__device__ inline T sym3_lmax(T a00, T a11, T a22, T a01, T a02, T a12) {
  const T q = (a00 + a11 + a22) / T(3);
  const T p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const T b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  const T p2 = b00 * b00 + b11 * b11 + b22 * b22 + T(2) * p1;
  if (!(p2 > T(0))) return q;
  const T p = sqrt(p2 / T(6));
  const T ip = T(1) / p;
  const T c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip,
          c12 = a12 * ip;
  T r = T(0.5) * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) +
                  c02 * (c01 * c12 - c11 * c02));
  r = r < T(-1) ? T(-1) : (r > T(1) ? T(1) : r);
  const T phi = acos(r) / T(3);
  return q + T(2) * p * cos(phi);
}

// rho * acoustic tensor n . (d sigma / d eps) . n of the CDM law (symmetric)
template <class T>
__device__ inline void acoustic_rhoQ(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law,
                                     T Q[3][3]) {
  Parts<T> p = cdm_parts(u, law);
  const T agr = p.ac * m.gr;
  const T h = (m.mu + p.ac * m.xi0 * m.gr) - T(0.5) * agr * p.xi;
  // (eps n) of the scaled strain; the eps/sqrt(I2) terms are scale free
  const T im = p.im;
  const T en[3] = {(u[0] * n[0] + u[3] * n[1] + u[5] * n[2]) * im,
                   (u[3] * n[0] + u[1] * n[1] + u[4] * n[2]) * im,
                   (u[5] * n[0] + u[4] * n[1] + u[2] * n[2]) * im};
  const T is = p.guard ? T(0) : T(1) / p.sp;
  const T c1 = agr * is;                       // coefficient of n (eps n) + (eps n) n
  const T c2 = agr * p.I1p * is * is * is;     // coefficient of (eps n)(eps n)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      Q[i][k] = m.lam * n[i] * n[k] + h * ((i == k ? T(1) : T(0)) + n[i] * n[k]) -
                c1 * (n[i] * en[k] + en[i] * n[k]) + c2 * en[i] * en[k];
}

template <class T>
__device__ inline T llf_speed(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law) {
  T Q[3][3];
  acoustic_rhoQ(u, n, m, law, Q);
  T lm = sym3_lmax(Q[0][0], Q[1][1], Q[2][2], Q[0][1], Q[0][2], Q[1][2]) / m.rho;
  return lm > T(0) ? sqrt(lm) : T(0);
}

// Pointwise functions of the continuum-damage law
struct CdmLaw {
  template <class T>
  __device__ static void stress(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
    cdm_stress(u, m, law, sig);
  }
  template <class T>
  __device__ static T stress_rate(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
    return cdm_stress_rate(u, m, law, sig);
  }
  template <class T>
  __device__ static T rate(const T* u, const MatP<T>& m, const Law<T>& law) {
    return cdm_rate(u, m, law);
  }
  template <class T>
  __device__ static void tangent(const T* u, const MatP<T>& m, const Law<T>& law, T ds[6][7]) {
    cdm_tangent(u, m, law, ds);
  }
  template <class T>
  __device__ static T speed(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law) {
    return llf_speed(u, n, m, law);
  }
  // effective Lame parameters on boundaries (Eq. effective-cdb)
  template <class T>
  __device__ static void lame(const T* u, const MatP<T>& m, const Law<T>& law, T& lam, T& mu) {
    Parts<T> p = cdm_parts(u, law);
    lam = m.lam - p.ac * m.gr * p.xi / T(3);
    mu = m.mu + p.ac * m.xi0 * m.gr - T(0.5) * p.ac * m.gr * p.xi;
  }
};

// Internal-variable law with the Murnaghan terms off (Eq. ivm-model):
//   sigma = (1 - alpha)(lambda0 I1 delta + 2 mu0 eps),
//   r = [lambda0 I1^2 / 2 + mu0 I2 - gamma_b (alpha / (1 - alpha))^2] / (gamma_b tau_b),
// alpha clamped to [0, amax].  Material slots: gr = gamma_b,
// cd = 1 / (gamma_b tau_b) (xi0 unused).
struct IvmLaw {
  template <class T> struct Pt {
    T I1, I2, g, ac, dac;
  };
  template <class T>
  __device__ static Pt<T> parts(const T* u, const Law<T>& law) {
    Pt<T> p;
    p.I1 = u[0] + u[1] + u[2];
    p.I2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] +
           T(2) * (u[3] * u[3] + u[4] * u[4] + u[5] * u[5]);
    const T a = u[9];
    p.ac = a < T(0) ? T(0) : (a > law.amax ? law.amax : a);
    p.dac = (a >= T(0) && a <= law.amax) ? T(1) : T(0);
    p.g = T(1) - p.ac;
    return p;
  }
  template <class T>
  __device__ static void stress_p(const Pt<T>& p, const T* u, const MatP<T>& m, T sig[6]) {
    const T c = T(2) * m.mu * p.g, iso = m.lam * p.g * p.I1;
#pragma unroll
    for (int k = 0; k < 6; ++k) sig[k] = c * u[k] + (k < 3 ? iso : T(0));
  }
  template <class T>
  __device__ static T rate_p(const Pt<T>& p, const MatP<T>& m) {
    const T q = p.ac / p.g;
    return m.cd * (T(0.5) * m.lam * p.I1 * p.I1 + m.mu * p.I2 - m.gr * q * q);
  }
  template <class T>
  __device__ static void stress(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
    stress_p(parts(u, law), u, m, sig);
  }
  template <class T>
  __device__ static T stress_rate(const T* u, const MatP<T>& m, const Law<T>& law, T sig[6]) {
    const Pt<T> p = parts(u, law);
    stress_p(p, u, m, sig);
    return rate_p(p, m);
  }
  template <class T>
  __device__ static T rate(const T* u, const MatP<T>& m, const Law<T>& law) {
    return rate_p(parts(u, law), m);
  }
  // d sigma_k / d u_q (q < 6 strain entries, q = 6 alpha)
  template <class T>
  __device__ static void tangent(const T* u, const MatP<T>& m, const Law<T>& law, T ds[6][7]) {
    const Pt<T> p = parts(u, law);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
      for (int q = 0; q < 6; ++q)
        ds[k][q] = p.g * ((k == q ? T(2) * m.mu : T(0)) + (k < 3 && q < 3 ? m.lam : T(0)));
      ds[k][6] = -p.dac * (T(2) * m.mu * u[k] + (k < 3 ? m.lam * p.I1 : T(0)));
    }
  }
  // the acoustic tensor is that of the damaged isotropic moduli
  template <class T>
  __device__ static T speed(const T* u, const T n[3], const MatP<T>& m, const Law<T>& law) {
    const Pt<T> p = parts(u, law);
    return sqrt(p.g * (m.lam + T(2) * m.mu) / m.rho);
  }
  // effective Lame parameters on boundaries (Eq. effective-ivm)
  template <class T>
  __device__ static void lame(const T* u, const MatP<T>& m, const Law<T>& law, T& lam, T& mu) {
    const Pt<T> p = parts(u, law);
    lam = p.g * m.lam;
    mu = p.g * m.mu;
  }
};

template <class T>
__device__ inline bool same_material(const MatP<T>& a, const MatP<T>& b) {
  return a.rho == b.rho && a.lam == b.lam && a.mu == b.mu && a.gr == b.gr && a.xi0 == b.xi0 &&
         a.cd == b.cd;
}

// Local Lax-Friedrichs flux at one face point
template <class LW = CdmLaw, class T>
__device__ inline void llf_flux(const T* um, const T* up, const T n[3], const MatP<T>& mm,
                                const MatP<T>& mp, const Law<T>& law, T F[10]) {
  T Fm[10], Fp[10], ub[10];
  normal_flux<LW>(um, n, mm, law, Fm);
  normal_flux<LW>(up, n, mp, law, Fp);
#pragma unroll
  for (int k = 0; k < 10; ++k) ub[k] = T(0.5) * (um[k] + up[k]);
  // the speed at the mean state is the same for equal materials
  const T c1 = LW::speed(ub, n, mm, law);
  T C = c1;
  if (!same_material(mm, mp)) {
    const T c2 = LW::speed(ub, n, mp, law);
    C = c1 > c2 ? c1 : c2;
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) F[k] = T(0.5) * (Fm[k] + Fp[k]) + T(0.5) * C * (um[k] - up[k]);
}

template <class T>
__device__ inline void face_frame(const T n[3], T s[3], T t[3]) {
  const T ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
  int k = 0;
  if (ay < ax) k = 1;
  if (az < (k == 0 ? ax : ay)) k = 2;
  T e[3] = {T(0), T(0), T(0)};
  e[k] = T(1);
  s[0] = n[1] * e[2] - n[2] * e[1];
  s[1] = n[2] * e[0] - n[0] * e[2];
  s[2] = n[0] * e[1] - n[1] * e[0];
  const T il = T(1) / sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  s[0] *= il;
  s[1] *= il;
  s[2] *= il;
  t[0] = n[1] * s[2] - n[2] * s[1];
  t[1] = n[2] * s[0] - n[0] * s[2];
  t[2] = n[0] * s[1] - n[1] * s[0];
}

// free surface (kind 1) or absorbing (kind 2) boundary flux from the interior trace
template <class LW = CdmLaw, class T>
__device__ inline void boundary_flux(int kind, const T* u, const T n[3], const MatP<T>& m,
                                     const Law<T>& law, T F[10]) {
  T lam, mu;
  LW::lame(u, m, law, lam, mu);
  T s[3], t[3];
  face_frame(n, s, t);
  auto epsv = [&](const T* a, T out[3]) {
    out[0] = u[0] * a[0] + u[3] * a[1] + u[5] * a[2];
    out[1] = u[3] * a[0] + u[1] * a[1] + u[4] * a[2];
    out[2] = u[5] * a[0] + u[4] * a[1] + u[2] * a[2];
  };
  auto dot = [](const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  T en[3], es[3], et[3];
  epsv(n, en);
  epsv(s, es);
  epsv(t, et);
  const T enn = dot(n, en), ess = dot(s, es), ett = dot(t, et), ens = dot(s, en), etn = dot(t, en);
  const T vn = dot(u + 6, n), vs = dot(u + 6, s), vt = dot(u + 6, t);
  const T M = lam + T(2) * mu;
  const T snn = M * enn + lam * (ess + ett);
  const T cp = sqrt(M / m.rho), cs = sqrt(mu / m.rho);
  T b[3], fv[3];
  if (kind == 1) {
    const T bn = vn - snn / M * cp, bs = vs - T(2) * ens * cs, bt = vt - T(2) * etn * cs;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      b[i] = bn * n[i] + bs * s[i] + bt * t[i];
      fv[i] = T(0);
    }
  } else {
    const T an = T(0.5) * (vn - cp * snn / M), as = T(0.5) * vs - cs * ens,
            at = T(0.5) * vt - cs * etn;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      b[i] = an * n[i] + as * s[i] + at * t[i];
      fv[i] = cp * an * n[i] + cs * as * s[i] + cs * at * t[i];
    }
  }
  F[0] = -b[0] * n[0];
  F[1] = -b[1] * n[1];
  F[2] = -b[2] * n[2];
  F[3] = T(-0.5) * (b[0] * n[1] + b[1] * n[0]);
  F[4] = T(-0.5) * (b[1] * n[2] + b[2] * n[1]);
  F[5] = T(-0.5) * (b[2] * n[0] + b[0] * n[2]);
  F[6] = fv[0];
  F[7] = fv[1];
  F[8] = fv[2];
  F[9] = T(0);
}

// strain-energy density W (FP64 diagnostics)
__device__ inline double cdm_energy(const double* u, const MatP<double>& m,
                                    const Law<double>& law) {
  Parts<double> p = cdm_parts(u, law);
  return 0.5 * m.lam * p.I1 * p.I1 + (m.mu + p.ac * m.xi0 * m.gr) * p.I2 -
         p.ac * m.gr * p.I1 * p.s;
}

}  // namespace dgd
