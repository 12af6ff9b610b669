"""Orthonormal Dubiner basis on the reference tetrahedron (oracle).

The paper approximates each conservative variable inside an element by a
modal expansion in Dubiner's orthogonal polynomials, L = (p+1)(p+2)(p+3)/6
functions for degree p (Section 2.2, Eq. modal dg space).  The paper does not
fix the normalisation or the ordering; the reading used here (shared with the
library interface) is:

* reference tetrahedron T = {xi >= 0, xi1 + xi2 + xi3 <= 1};
* psi_ijk = P_i^(0,0)(a) ((1-b)/2)^i P_j^(2i+1,0)(b) ((1-c)/2)^(i+j)
  P_k^(2i+2j+2,0)(c) with collapsed coordinates a = 2 xi1/(1-xi2-xi3) - 1,
  b = 2 xi2/(1-xi3) - 1, c = 2 xi3 - 1;
* phi_ijk = psi_ijk sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3)), so that the reference
  mass matrix is the identity;
* modes ordered by total degree i+j+k, then lexicographically by (i, j, k).

The oracle expands every phi into monomials xi1^a xi2^b xi3^c with exact
rational coefficients (Python fractions), using the explicit sum formula of
the Jacobi polynomials.  Values and gradients are then plain monomial sums,
and exact integrals over T follow from  int x^a y^b z^c = a! b! c!/(a+b+c+3)!.
"""
from fractions import Fraction
from functools import lru_cache
from math import comb, factorial, sqrt

import numpy as np
import torch

DT = torch.float64


def n_modes(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def mode_indices(N):
    """(i, j, k) triples in the library's mode order."""
    idx = [(i, j, k) for i in range(N + 1) for j in range(N + 1)
           for k in range(N + 1) if i + j + k <= N]
    idx.sort(key=lambda t: (t[0] + t[1] + t[2], t[0], t[1], t[2]))
    return idx


# --- exact polynomials in three variables: {(a, b, c): Fraction} -------------

def _padd(p, q, s=1):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, Fraction(0)) + s * v
        if out[k] == 0:
            del out[k]
    return out


def _pmul(p, q):
    out = {}
    for (a1, b1, c1), v1 in p.items():
        for (a2, b2, c2), v2 in q.items():
            k = (a1 + a2, b1 + b2, c1 + c2)
            out[k] = out.get(k, Fraction(0)) + v1 * v2
    return {k: v for k, v in out.items() if v != 0}


def _ppow(p, n):
    out = {(0, 0, 0): Fraction(1)}
    for _ in range(n):
        out = _pmul(out, p)
    return out


def _pscale(p, s):
    return {k: v * s for k, v in p.items() if v * s != 0}


def jacobi_coeffs(n, alpha):
    """Monomial coefficients of P_n^(alpha,0)(t) from the explicit sum
    P_n^(a,b)(t) = sum_s C(n+a, n-s) C(n+b, s) ((t-1)/2)^s ((t+1)/2)^(n-s)."""
    # univariate polynomials as lists of Fractions
    def umul(p, q):
        r = [Fraction(0)] * (len(p) + len(q) - 1)
        for i, a in enumerate(p):
            for j, b in enumerate(q):
                r[i + j] += a * b
        return r

    def upow(p, k):
        r = [Fraction(1)]
        for _ in range(k):
            r = umul(r, p)
        return r

    tm = [Fraction(-1, 2), Fraction(1, 2)]   # (t-1)/2
    tp = [Fraction(1, 2), Fraction(1, 2)]    # (t+1)/2
    out = [Fraction(0)] * (n + 1)
    for s in range(n + 1):
        c = comb(n + alpha, n - s) * comb(n, s)
        term = umul(upow(tm, s), upow(tp, n - s))
        for m, v in enumerate(term):
            out[m] += c * v
    return out


@lru_cache(maxsize=None)
def _psi_exact(i, j, k):
    """psi_ijk as an exact polynomial in (xi1, xi2, xi3)."""
    one = {(0, 0, 0): Fraction(1)}
    x = {(1, 0, 0): Fraction(1)}
    y = {(0, 1, 0): Fraction(1)}
    z = {(0, 0, 1): Fraction(1)}
    w1 = _padd(_padd(one, y, -1), z, -1)                 # 1 - y - z
    l1 = _padd(_padd(_padd(_pscale(x, 2), y), z), one, -1)  # 2x - 1 + y + z
    w2 = _padd(one, z, -1)                                # 1 - z
    l2 = _padd(_padd(_pscale(y, 2), z), one, -1)          # 2y - 1 + z
    l3 = _padd(_pscale(z, 2), one, -1)                    # 2z - 1
    # P_i(a) (1-y-z)^i, with a (1-y-z) = 2x - 1 + y + z
    A = {}
    for m, cm in enumerate(jacobi_coeffs(i, 0)):
        if cm != 0:
            A = _padd(A, _pscale(_pmul(_ppow(l1, m), _ppow(w1, i - m)), cm))
    # P_j^(2i+1,0)(b) (1-z)^j, with b (1-z) = 2y - 1 + z
    B = {}
    for m, cm in enumerate(jacobi_coeffs(j, 2 * i + 1)):
        if cm != 0:
            B = _padd(B, _pscale(_pmul(_ppow(l2, m), _ppow(w2, j - m)), cm))
    # P_k^(2i+2j+2,0)(c), c = 2z - 1
    C = {}
    for m, cm in enumerate(jacobi_coeffs(k, 2 * i + 2 * j + 2)):
        if cm != 0:
            C = _padd(C, _pscale(_ppow(l3, m), cm))
    return _pmul(_pmul(A, B), C)


def norm_factor(i, j, k):
    """phi = psi * sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3))."""
    return sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))


def psi_exact(i, j, k):
    return dict(_psi_exact(i, j, k))


def exact_monomial_integral(a, b, c):
    """int_T xi1^a xi2^b xi3^c = a! b! c! / (a+b+c+3)!  (exact rational)."""
    return Fraction(factorial(a) * factorial(b) * factorial(c),
                    factorial(a + b + c + 3))


def exact_integral(p):
    return sum((v * exact_monomial_integral(*k) for k, v in p.items()),
               Fraction(0))


def derivative(p, axis):
    out = {}
    for k, v in p.items():
        if k[axis] > 0:
            kk = list(k)
            kk[axis] -= 1
            out[tuple(kk)] = out.get(tuple(kk), Fraction(0)) + v * k[axis]
    return out


class Basis:
    """Values and gradients of the orthonormal basis of degree N at points."""

    def __init__(self, N):
        self.N = N
        self.L = n_modes(N)
        self.modes = mode_indices(N)
        self.monos = [(a, b, c) for a in range(N + 1) for b in range(N + 1)
                      for c in range(N + 1) if a + b + c <= N]
        mi = {m: t for t, m in enumerate(self.monos)}
        coef = np.zeros((self.L, len(self.monos)))
        dcoef = np.zeros((3, self.L, len(self.monos)))
        for l, (i, j, k) in enumerate(self.modes):
            p = _psi_exact(i, j, k)
            s = norm_factor(i, j, k)
            for mono, v in p.items():
                coef[l, mi[mono]] = float(v) * s
            for ax in range(3):
                for mono, v in derivative(p, ax).items():
                    dcoef[ax, l, mi[mono]] = float(v) * s
        self.coef = torch.tensor(coef, dtype=DT)
        self.dcoef = torch.tensor(dcoef, dtype=DT)
        self.pows = torch.tensor(self.monos, dtype=DT)

    def _mono(self, xi):
        xi = torch.as_tensor(xi, dtype=DT)
        return torch.prod(xi[..., None, :] ** self.pows, dim=-1)   # (..., nmono)

    def values(self, xi):
        """phi_l(xi) for points xi (..., 3) -> (..., L)."""
        return self._mono(xi) @ self.coef.T

    def gradients(self, xi):
        """d phi_l / d xi_e at points (..., 3) -> (..., 3, L)."""
        m = self._mono(xi)
        return torch.stack([m @ self.dcoef[e].T for e in range(3)], dim=-2)
