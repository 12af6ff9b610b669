// Host-side reference-element generator (FP64).  See refgen.hpp.
#include "refgen.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <tuple>

namespace dgd {

const int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
const int kFaceVerts[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};

int n_modes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }

// P_n^(a,b)(x) and its derivative by the three-term recurrence;
// d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1).
static double jacobi(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * ((a - b) + (a + b + 2.0) * x);
  for (int k = 2; k <= n; ++k) {
    double c = 2.0 * k + a + b;
    double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    double a2 = (c - 1.0) * (c * (c - 2.0) * x + a * a - b * b);
    double a3 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    double p2 = (a2 * p1 - a3 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

static double djacobi(int n, double a, double b, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

void gauss_jacobi(int n, double alpha, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    // Chebyshev-like start, refined by Newton with deflation of found roots
    double x = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    if (k > 0 && x <= t[k - 1]) x = 0.5 * (t[k - 1] + 1.0);
    for (int it = 0; it < 200; ++it) {
      double p = jacobi(n, alpha, 0.0, x);
      double dp = djacobi(n, alpha, 0.0, x);
      double defl = 0.0;
      for (int j = 0; j < k; ++j) defl += 1.0 / (x - t[j]);
      double dx = p / (dp - p * defl);
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[k] = x;
  }
  std::sort(t.begin(), t.end());
  for (int k = 0; k < n; ++k) {
    double dp = djacobi(n, alpha, 0.0, t[k]);
    w[k] = std::pow(2.0, alpha + 1.0) / ((1.0 - t[k] * t[k]) * dp * dp);
  }
}

struct Mode { int i, j, k; };

static std::vector<Mode> modes(int N) {
  std::vector<Mode> m;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; i + j <= N; ++j)
      for (int k = 0; i + j + k <= N; ++k) m.push_back({i, j, k});
  std::sort(m.begin(), m.end(), [](const Mode& A, const Mode& B) {
    return std::make_tuple(A.i + A.j + A.k, A.i, A.j, A.k) <
           std::make_tuple(B.i + B.j + B.k, B.i, B.j, B.k);
  });
  return m;
}

static double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

void basis_eval(int N, const double xi[3], double* phi, double* dphi) {
  const double x = xi[0], y = xi[1], z = xi[2];
  const double omyz = 1.0 - y - z, omz = 1.0 - z;
  const double a = 2.0 * x / omyz - 1.0, b = 2.0 * y / omz - 1.0, c = 2.0 * z - 1.0;
  const double hb = 0.5 * (1.0 - b), hc = 0.5 * (1.0 - c);
  std::vector<Mode> ms = modes(N);
  const int L = (int)ms.size();
  for (int l = 0; l < L; ++l) {
    const int i = ms[l].i, j = ms[l].j, k = ms[l].k;
    const double nrm = std::sqrt((2.0 * i + 1.0) * (2.0 * i + 2.0 * j + 2.0) *
                                 (2.0 * i + 2.0 * j + 2.0 * k + 3.0));
    const double fa = jacobi(i, 0.0, 0.0, a);
    const double gb = jacobi(j, 2.0 * i + 1.0, 0.0, b);
    const double hcv = jacobi(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
    const double Bv = ipow(hb, i) * gb;
    const double Cv = ipow(hc, i + j) * hcv;
    phi[l] = nrm * fa * Bv * Cv;
    if (dphi) {
      const double dfa = djacobi(i, 0.0, 0.0, a);
      const double dgb = djacobi(j, 2.0 * i + 1.0, 0.0, b);
      const double dhc = djacobi(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
      const double Bp = (i > 0 ? -0.5 * i * ipow(hb, i - 1) * gb : 0.0) + ipow(hb, i) * dgb;
      const double Cp = (i + j > 0 ? -0.5 * (i + j) * ipow(hc, i + j - 1) * hcv : 0.0) +
                        ipow(hc, i + j) * dhc;
      const double pa = dfa * Bv * Cv, pb = fa * Bp * Cv, pc = fa * Bv * Cp;
      // a(x,y,z), b(y,z), c(z): chain rule
      const double dx = pa * 2.0 / omyz;
      const double dy = pa * (1.0 + a) / omyz + pb * 2.0 / omz;
      const double dz = pa * (1.0 + a) / omyz + pb * (1.0 + b) / omz + pc * 2.0;
      dphi[0 * L + l] = nrm * dx;
      dphi[1 * L + l] = nrm * dy;
      dphi[2 * L + l] = nrm * dz;
    }
  }
}

static const double kRefVerts[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

RefData build_reference(int N) {
  if (N < 1 || N > 6) throw std::invalid_argument("degree out of range");
  RefData r;
  r.N = N;
  r.L = n_modes(N);
  const int n = N + 1;
  r.Q = n * n * n;
  r.Ns = n * n;
  r.Nt = n;
  std::vector<double> ta, wa, tb, wb, tc, wc;
  gauss_jacobi(n, 0.0, ta, wa);
  gauss_jacobi(n, 1.0, tb, wb);
  gauss_jacobi(n, 2.0, tc, wc);
  for (int ia = 0; ia < n; ++ia)
    for (int ib = 0; ib < n; ++ib)
      for (int ic = 0; ic < n; ++ic) {
        const double A = ta[ia], B = tb[ib], C = tc[ic];
        r.xq.push_back((1 + A) * (1 - B) * (1 - C) / 8.0);
        r.xq.push_back((1 + B) * (1 - C) / 4.0);
        r.xq.push_back((1 + C) / 2.0);
        r.wq.push_back(wa[ia] * wb[ib] * wc[ic] / 64.0);
      }
  for (int ia = 0; ia < n; ++ia)
    for (int ib = 0; ib < n; ++ib) {
      r.eta.push_back((1 + ta[ia]) * (1 - tb[ib]) / 4.0);
      r.eta.push_back((1 + tb[ib]) / 2.0);
      r.beta.push_back(wa[ia] * wb[ib] / 4.0);
    }
  for (int z = 0; z < n; ++z) {
    r.tau.push_back(0.5 * (1.0 + ta[z]));
    r.gamma.push_back(0.5 * wa[z]);
  }
  const int L = r.L, Q = r.Q, Ns = r.Ns;
  r.V.assign((size_t)Q * L, 0.0);
  r.Pw.assign((size_t)L * Q, 0.0);
  r.Sw.assign((size_t)3 * L * Q, 0.0);
  r.K.assign((size_t)3 * L * L, 0.0);
  std::vector<double> phi(L), dphi(3 * L);
  for (int q = 0; q < Q; ++q) {
    basis_eval(N, &r.xq[3 * q], phi.data(), dphi.data());
    for (int l = 0; l < L; ++l) {
      r.V[(size_t)q * L + l] = phi[l];
      r.Pw[(size_t)l * Q + q] = r.wq[q] * phi[l];
      for (int e = 0; e < 3; ++e) r.Sw[((size_t)e * L + l) * Q + q] = r.wq[q] * dphi[e * L + l];
    }
    for (int e = 0; e < 3; ++e)
      for (int k = 0; k < L; ++k)
        for (int l = 0; l < L; ++l)
          r.K[((size_t)e * L + k) * L + l] += r.wq[q] * phi[k] * dphi[e * L + l];
  }
  r.F.assign((size_t)4 * 6 * Ns * L, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int s = 0; s < 6; ++s)
      for (int i = 0; i < Ns; ++i) {
        const double e1 = r.eta[2 * i], e2 = r.eta[2 * i + 1];
        const double bary[3] = {1.0 - e1 - e2, e1, e2};
        double loc[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j) loc[kPerm3[s][j]] = bary[j];
        double xi[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j)
          for (int d = 0; d < 3; ++d) xi[d] += loc[j] * kRefVerts[kFaceVerts[f][j]][d];
        basis_eval(N, xi, phi.data(), nullptr);
        for (int l = 0; l < L; ++l) r.F[(((size_t)f * 6 + s) * Ns + i) * L + l] = phi[l];
      }
  // strong-form derivative of a projected field: KP[e] = K[e] Pw
  r.KP.assign((size_t)3 * L * Q, 0.0);
  for (int e = 0; e < 3; ++e)
    for (int k = 0; k < L; ++k)
      for (int l = 0; l < L; ++l) {
        const double kk = r.K[((size_t)e * L + k) * L + l];
        for (int q = 0; q < Q; ++q) r.KP[((size_t)e * L + k) * Q + q] += kk * r.Pw[(size_t)l * Q + q];
      }
  // Om[z][j] = int_0^{tau_z} l_j(s) ds for the Lagrange polynomials l_j of the
  // time points (monomial coefficients built factor by factor)
  r.Om.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    std::vector<double> c(1, 1.0);
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      const double d = r.tau[j] - r.tau[k];
      std::vector<double> nc(c.size() + 1, 0.0);
      for (size_t i = 0; i < c.size(); ++i) {
        nc[i + 1] += c[i] / d;
        nc[i] -= c[i] * r.tau[k] / d;
      }
      c.swap(nc);
    }
    for (int z = 0; z < n; ++z) {
      double acc = 0.0, pw = r.tau[z];
      for (size_t i = 0; i < c.size(); ++i) {
        acc += c[i] / (double)(i + 1) * pw;
        pw *= r.tau[z];
      }
      r.Om[(size_t)z * n + j] = acc;
    }
  }
  std::vector<Mode> ms = modes(N);
  for (auto& m : ms) r.deg.push_back(m.i + m.j + m.k);
  return r;
}

}  // namespace dgd
