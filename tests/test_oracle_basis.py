"""Pins of the oracle's basis, quadrature and reference matrices.

Each check ties the oracle to something other than itself: exact rational
integrals over the reference tetrahedron (int x^a y^b z^c = a!b!c!/(a+b+c+3)!),
the collapsed-coordinate definition of the Dubiner basis evaluated with
scipy's Jacobi polynomials, finite differences, and polynomial-degree
structure.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest
import torch
from scipy.special import eval_jacobi

from oracle import basis as B
from oracle.quadrature import face_rule, time_rule, volume_rule
from oracle.refmat import RefElement, face_to_ref


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_volume_rule_exact_to_2N_plus_1(N):
    x, w = volume_rule(N)
    assert x.shape[0] == (N + 1) ** 3
    for a in range(2 * N + 2):
        for b in range(2 * N + 2 - a):
            for c in range(2 * N + 2 - a - b):
                exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
                got = float((w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c).sum())
                assert abs(got - exact) <= 1e-15 + 1e-13 * exact


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_face_and_time_rules(N):
    eta, beta = face_rule(N)
    assert abs(float(beta.sum()) - 1.0) < 1e-14
    for a in range(2 * N + 2):
        for b in range(2 * N + 2 - a):
            # int_tri x^a y^b = a! b! / (a+b+2)!, area 1/2
            exact = 2.0 * factorial(a) * factorial(b) / factorial(a + b + 2)
            got = float((beta * eta[:, 0] ** a * eta[:, 1] ** b).sum())
            assert abs(got - exact) < 1e-14
    tau, gamma = time_rule(N)
    for k in range(2 * N + 2):
        assert abs(float((gamma * tau ** k).sum()) - 1.0 / (k + 1)) < 1e-14


@pytest.mark.parametrize("N", [1, 2, 3])
def test_basis_orthonormal_exactly(N):
    modes = B.mode_indices(N)
    assert len(modes) == B.n_modes(N)
    for a, ma in enumerate(modes):
        pa = B.psi_exact(*ma)
        for b, mb in enumerate(modes[: a + 1]):
            pb = B.psi_exact(*mb)
            val = B.exact_integral(B._pmul(pa, pb))
            if a == b:
                i, j, k = ma
                assert val == Fraction(1, (2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
            else:
                assert val == 0


def _collapsed(N, xi):
    """Definition of the basis through collapsed coordinates (scipy Jacobi)."""
    x, y, z = xi[:, 0], xi[:, 1], xi[:, 2]
    a = 2 * x / (1 - y - z) - 1
    b = 2 * y / (1 - z) - 1
    c = 2 * z - 1
    out = []
    for (i, j, k) in B.mode_indices(N):
        v = (eval_jacobi(i, 0, 0, a) * ((1 - b) / 2) ** i
             * eval_jacobi(j, 2 * i + 1, 0, b) * ((1 - c) / 2) ** (i + j)
             * eval_jacobi(k, 2 * i + 2 * j + 2, 0, c))
        out.append(v * B.norm_factor(i, j, k))
    return np.stack(out, -1)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_basis_matches_collapsed_definition(N):
    rng = np.random.default_rng(1)
    p = rng.random((200, 4))
    p /= p.sum(1, keepdims=True)
    xi = p[:, 1:]
    ref = B.Basis(N)
    got = ref.values(xi).numpy()
    assert np.allclose(got, _collapsed(N, xi), rtol=0, atol=1e-11)


@pytest.mark.parametrize("N", [2, 4])
def test_gradients_finite_difference(N):
    rng = np.random.default_rng(2)
    p = rng.random((20, 4)) + 0.2
    p /= p.sum(1, keepdims=True)
    xi = torch.tensor(p[:, 1:])
    bas = B.Basis(N)
    g = bas.gradients(xi)
    h = 1e-6
    for e in range(3):
        d = torch.zeros(3, dtype=torch.float64)
        d[e] = h
        fd = (bas.values(xi + d) - bas.values(xi - d)) / (2 * h)
        assert torch.allclose(g[:, e, :], fd, atol=1e-6)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_reference_matrices(N):
    ref = RefElement(N)
    L = ref.L
    assert torch.allclose(ref.M, torch.eye(L, dtype=torch.float64), atol=1e-13)
    # K^e_kl = int phi_k dphi_l/dxi_e, exact rational integral of the expansion
    modes = ref.basis.modes
    for e in range(3):
        for k, mk in enumerate(modes):
            pk = B.psi_exact(*mk)
            for l, ml in enumerate(modes):
                pl = B.derivative(B.psi_exact(*ml), e)
                exact = float(B.exact_integral(B._pmul(pk, pl))) * \
                    B.norm_factor(*mk) * B.norm_factor(*ml)
                assert abs(float(ref.K[e, k, l]) - exact) < 1e-12
                # derivative lowers the degree: zero unless deg k < deg l
                if sum(mk) >= sum(ml):
                    assert abs(exact) < 1e-13
    # projection reproduces the basis
    assert torch.allclose(ref.P @ ref.V, torch.eye(L, dtype=torch.float64), atol=1e-13)


@pytest.mark.parametrize("N", [2, 3])
def test_face_trace_and_lift(N):
    ref = RefElement(N)
    # the four reference faces: xi3 = 0, xi2 = 0, xi1 = 0, xi1+xi2+xi3 = 1
    for f, (ax, val) in enumerate([(2, 0.0), (1, 0.0), (0, 0.0), (None, 1.0)]):
        xi = face_to_ref(f, ref.eta)
        if ax is None:
            assert torch.allclose(xi.sum(1), torch.ones(ref.Ns, dtype=torch.float64))
        else:
            assert torch.allclose(xi[:, ax], torch.zeros(ref.Ns, dtype=torch.float64))
        assert torch.allclose(ref.Fown[f], ref.basis.values(xi))
        assert torch.allclose(ref.Lift[f], (ref.beta[:, None] * ref.Fown[f]).T)
    # divergence theorem on the reference element for phi_k * phi_l products:
    # sum_f |S_f^ref| int_f phi_k phi_l n_e = int (dphi_k/dxi_e phi_l + phi_k dphi_l/dxi_e)
    areas = [0.5, 0.5, 0.5, np.sqrt(3) / 2]
    normals = torch.tensor([[0, 0, -1], [0, -1, 0], [-1, 0, 0],
                            [1 / np.sqrt(3)] * 3], dtype=torch.float64)
    for e in range(3):
        lhs = sum(areas[f] * normals[f, e] * ref.Lift[f] @ ref.Fown[f] for f in range(4))
        rhs = ref.Kstiff[e] + ref.K[e]
        assert torch.allclose(lhs, rhs, atol=1e-12)
