"""Quadrature rules (oracle).

The paper integrates the space-time face flux with surface weights beta_i and
time weights gamma_z (Appendix A.2, Eq. 2nd term) and evaluates volume terms
on nodal points (Eqs. 3rd term, rhs term) without naming the rules.  Reading
used here: collapsed-coordinate (Stroud conical product) Gauss-Jacobi rules
with N+1 points per direction, exact to degree 2N+1:

* volume: Q = (N+1)^3 points on T, weights sum to 1/6;
* face:   Ns = (N+1)^2 points on the reference triangle
  {eta >= 0, eta1 + eta2 <= 1}, weights beta_i normalised to sum 1 (so that
  int_face g dS = |S_f| sum_i beta_i g_i);
* time:   Nt = N+1 Gauss-Legendre points tau_z on [0, 1], weights gamma_z
  summing to 1.

Gauss-Jacobi nodes and weights come from scipy.special.roots_jacobi (weight
(1-t)^alpha on [-1, 1]).
"""
import numpy as np
import torch
from scipy.special import roots_jacobi

DT = torch.float64


def gauss_jacobi(n, alpha):
    t, w = roots_jacobi(n, alpha, 0.0)
    return np.asarray(t, dtype=np.float64), np.asarray(w, dtype=np.float64)


def volume_rule(N):
    """Points (Q, 3) and weights (Q,) on the reference tetrahedron."""
    n = N + 1
    ta, wa = gauss_jacobi(n, 0.0)
    tb, wb = gauss_jacobi(n, 1.0)
    tc, wc = gauss_jacobi(n, 2.0)
    pts, wts = [], []
    for a, wa_ in zip(ta, wa):
        for b, wb_ in zip(tb, wb):
            for c, wc_ in zip(tc, wc):
                x = (1 + a) * (1 - b) * (1 - c) / 8.0
                y = (1 + b) * (1 - c) / 4.0
                z = (1 + c) / 2.0
                pts.append((x, y, z))
                # dx dy dz = (1/64) (1-b) (1-c)^2 da db dc
                wts.append(wa_ * wb_ * wc_ / 64.0)
    return torch.tensor(pts, dtype=DT), torch.tensor(wts, dtype=DT)


def face_rule(N):
    """Points (Ns, 2) on the reference triangle and weights beta (sum 1)."""
    n = N + 1
    ta, wa = gauss_jacobi(n, 0.0)
    tb, wb = gauss_jacobi(n, 1.0)
    pts, wts = [], []
    for a, wa_ in zip(ta, wa):
        for b, wb_ in zip(tb, wb):
            pts.append(((1 + a) * (1 - b) / 4.0, (1 + b) / 2.0))
            # d eta1 d eta2 = (1/8)(1-b) da db; area 1/2 -> beta = 2 w
            wts.append(2.0 * wa_ * wb_ / 8.0)
    return torch.tensor(pts, dtype=DT), torch.tensor(wts, dtype=DT)


def time_rule(N):
    """Gauss-Legendre points tau (Nt,) on [0, 1] and weights gamma (sum 1)."""
    t, w = gauss_jacobi(N + 1, 0.0)
    return torch.tensor((1 + t) / 2.0, dtype=DT), torch.tensor(w / 2.0, dtype=DT)
