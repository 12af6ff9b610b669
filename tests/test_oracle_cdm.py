"""Pins of the oracle's pointwise CDM law, Jacobians and LLF constant.

* alpha = 0 reduces the CDM stress to Hooke's law (closed form);
* sigma is the strain derivative of the energy W and r_alpha = -C_d dW/dalpha
  above the threshold (finite differences);
* the flux Jacobians at alpha = 0 equal the effective matrices the paper
  prints (Appendix A.3, Eqs. matrix_Beff_1..3, after the typo readings);
* the LLF constant equals c_p at alpha = 0 and sqrt(lambda_max) of the
  acoustic tensor written out by hand, and reproduces the plane-wave speeds
  of the anisotropy verification (Section 3.3, Table 1) derived by hand.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cdm
from tests._golden import printed_matrices

DT = torch.float64
AM = 0.5


def _mat(**kw):
    base = dict(rho=2760.0, lambda0=32e9, mu0=32e9, gamma_r=37e9, xi0=-0.75, Cd=1e-2)
    base.update(kw)
    return {k: torch.tensor(v, dtype=DT) for k, v in base.items()}


def _rand_u(n, seed=0, amp=1e-4, alpha=None):
    g = torch.Generator().manual_seed(seed)
    u = amp * torch.randn(n, 10, generator=g, dtype=DT)
    u[:, 6:9] *= 1e4
    u[:, 9] = torch.rand(n, generator=g, dtype=DT) * 0.45 if alpha is None else alpha
    return u


def test_hooke_limit():
    u = _rand_u(50, alpha=0.0)
    m = _mat()
    s = cdm.stress(u, m, AM)
    I1 = u[:, 0] + u[:, 1] + u[:, 2]
    ref = 2 * 32e9 * u[:, :6]
    ref[:, :3] += 32e9 * I1[:, None]
    assert torch.allclose(s, ref, rtol=1e-14, atol=0)


def test_stress_is_energy_derivative():
    u = _rand_u(30, seed=1)
    m = _mat()
    s = cdm.stress(u, m, AM)
    h = 1e-10
    for q in range(6):
        d = torch.zeros(10, dtype=DT)
        d[q] = h
        fd = (cdm.energy_density(u + d, m, AM) - cdm.energy_density(u - d, m, AM)) / (2 * h)
        w = 1.0 if q < 3 else 2.0     # a shear entry of u stands for eps_ij and eps_ji
        assert torch.allclose(fd, w * s[:, q], rtol=2e-6, atol=1e-3)


def test_damage_rate_is_energy_release():
    u = _rand_u(40, seed=2)
    m = _mat()
    r = cdm.r_alpha(u, m, AM)
    h = 1e-7
    d = torch.zeros(10, dtype=DT)
    d[9] = h
    dW = (cdm.energy_density(u + d, m, AM) - cdm.energy_density(u - d, m, AM)) / (2 * h)
    I1, I2 = cdm.invariants(u)
    xi = I1 / torch.sqrt(I2)
    above = xi > -0.75
    assert above.any() and (~above).any()
    assert torch.allclose(r[above], -m["Cd"] * dW[above], rtol=1e-6)
    assert (r[~above] == 0).all()
    # zero strain: guarded branch
    z = torch.zeros(3, 10, dtype=DT)
    z[:, 9] = 0.3
    assert (cdm.r_alpha(z, m, AM) == 0).all()
    assert (cdm.stress(z, m, AM) == 0).all()


def _names(lam, mu, rho):
    return dict(lam=lam, mu=mu, rho=rho, cp=math.sqrt((lam + 2 * mu) / rho),
                cs=math.sqrt(mu / rho))


def test_jacobian_equals_printed_effective_matrices():
    lam, mu, rho = 32e9, 30e9, 2760.0
    pm = printed_matrices(_names(lam, mu, rho), which=("B1", "B2", "B3"))
    m = _mat(lambda0=lam, mu0=mu, rho=rho)
    # zero state: the whole 10x10 Jacobian is the printed effective matrix
    B0 = cdm.flux_jacobian(torch.zeros(1, 10, dtype=DT), m, AM)[0]
    for d, key in enumerate(("B1", "B2", "B3")):
        assert np.allclose(B0[d].numpy(), pm[key], rtol=1e-14, atol=1e-12)
    # strained but undamaged: equal outside the alpha column
    u = _rand_u(5, seed=3, alpha=0.0)
    Bu = cdm.flux_jacobian(u, m, AM)
    for d, key in enumerate(("B1", "B2", "B3")):
        assert np.allclose(Bu[:, d, :, :9].numpy(), pm[key][None, :, :9], rtol=1e-13, atol=1e-12)
    # the uncorrected print fails the same comparison (the readings matter)
    raw = printed_matrices(_names(lam, mu, rho), corrected=False, which=("B2",))
    assert not np.allclose(np.nan_to_num(raw["B2"]), pm["B2"])


def test_jacobian_finite_difference():
    u = _rand_u(10, seed=4)
    m = _mat()
    B = cdm.flux_jacobian(u, m, AM)
    for q in range(10):
        h = 1e-9 if q < 6 else (1e-5 if q < 9 else 1e-7)
        d = torch.zeros(10, dtype=DT)
        d[q] = h
        fd = (cdm.flux(u + d, m, AM) - cdm.flux(u - d, m, AM)) / (2 * h)
        scale = B[..., q].abs().max() + 1e-30
        assert (fd - B[..., q]).abs().max() / scale < 1e-5


def _acoustic(u, n, m):
    """Acoustic tensor Q_ik = n_j n_l dsigma_ij/deps_kl / rho written out by hand
    for the CDM law (derivative of the stress of Eq. cdb-model)."""
    e = u[:6]
    eps = torch.tensor([[e[0], e[3], e[5]], [e[3], e[1], e[4]], [e[5], e[4], e[2]]], dtype=DT)
    I1 = float(e[0] + e[1] + e[2])
    I2 = float((eps * eps).sum())
    s = math.sqrt(I2)
    xi = I1 / s
    a = min(max(float(u[9]), 0.0), AM)
    lam, mu, gr, xi0, rho = (float(m[k]) for k in ("lambda0", "mu0", "gamma_r", "xi0", "rho"))
    en = eps @ n
    nn = torch.outer(n, n)
    Q = (lam * nn + 0.5 * (2 * (mu + a * xi0 * gr) - a * gr * xi) * (torch.eye(3, dtype=DT) + nn)
         - a * gr / s * (torch.outer(n, en) + torch.outer(en, n))
         + a * gr * I1 / s ** 3 * torch.outer(en, en))
    return Q / rho


def test_llf_speed():
    m = _mat()
    n = torch.tensor([[0.48, -0.6, 0.64]], dtype=DT)
    u0 = _rand_u(1, seed=5, alpha=0.0)
    c = cdm.llf_speed(u0, n, m, AM)
    assert abs(float(c) - math.sqrt(96e9 / 2760.0)) < 1e-9 * float(c)
    for seed in range(6):
        u = _rand_u(1, seed=10 + seed)
        c = float(cdm.llf_speed(u, n, m, AM))
        lmax = float(np.linalg.eigvalsh(_acoustic(u[0], n[0], m).numpy()).max())
        assert abs(c - math.sqrt(lmax)) < 1e-10 * c


@pytest.mark.parametrize("phi_deg", [0.0, 45.0, 90.0])
def test_anisotropy_speeds(phi_deg):
    """Section 3.3 / Table 1: alpha = 0.5, pre-strain diag(1e-3, 0, 0) rotated by
    phi about z, wavefront normal x.  The eigenvalues of B_1 at that state are
    +-(P, S, qS speeds).  Reference speeds come from the acoustic tensor
    written out by hand (above), evaluated with numpy."""
    m = _mat(Cd=0.0)
    ph = math.radians(phi_deg)
    Rz = torch.tensor([[math.cos(ph), -math.sin(ph), 0], [math.sin(ph), math.cos(ph), 0], [0, 0, 1]], dtype=DT)
    eps = Rz @ torch.diag(torch.tensor([1e-3, 0, 0], dtype=DT)) @ Rz.T
    u = torch.zeros(10, dtype=DT)
    u[:6] = torch.stack([eps[0, 0], eps[1, 1], eps[2, 2], eps[0, 1], eps[1, 2], eps[2, 0]])
    u[9] = 0.5
    n = torch.tensor([1.0, 0, 0], dtype=DT)
    Bn = cdm.normal_jacobian(u[None], n[None], m, AM)[0]
    ev = np.sort(np.linalg.eigvals(Bn.numpy()).real)
    want = np.sqrt(np.linalg.eigvalsh(_acoustic(u, n, m).numpy()))
    assert np.allclose(ev[-3:], np.sort(want), rtol=1e-9)
    if phi_deg == 0.0:
        # by hand: along x, rho c^2 = lambda0 + 2 mu' - 2 a gr + a gr xi - ... = 31.25 GPa,
        # transverse rho c^2 = mu0 + a xi0 gr - a gr / 2 = 8.875 GPa
        assert np.allclose(np.sort(want), np.sqrt(np.array([8.875e9, 8.875e9, 31.25e9]) / 2760.0), rtol=1e-12)
