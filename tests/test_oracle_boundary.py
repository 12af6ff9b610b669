"""Pins of the oracle's boundary fluxes (Appendix A.3).

* the printed eigenvector matrix R diagonalises the printed (corrected)
  B^{1,eff} with the printed Lambda (Eq. matrix-R);
* the oracle's T matches the printed rotation (Eq. matrix-T) and rotates a
  strain tensor as R eps' R^T does;
* the free-surface state is traction free and the flux has the closed form
  -sym(v^b (x) n) in the strain rows and zero in the velocity rows;
* the absorbing flux passes an outgoing characteristic unchanged and
  annihilates an incoming one.
"""
import math

import numpy as np
import torch

from oracle import boundary as bd
from tests._golden import printed_matrices

DT = torch.float64
AM = 0.5


def _frame_names(n, s, t):
    return dict(nx=n[0], ny=n[1], nz=n[2], sx=s[0], sy=s[1], sz=s[2],
                tx=t[0], ty=t[1], tz=t[2])


def test_printed_R_diagonalises_B1():
    lam, mu, rho = 20e9, 11e9, 2500.0
    names = dict(lam=lam, mu=mu, rho=rho, cp=math.sqrt((lam + 2 * mu) / rho),
                 cs=math.sqrt(mu / rho))
    pm = printed_matrices(names, which=("B1", "R"))
    cp, cs = names["cp"], names["cs"]
    Lam = np.diag([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp, 0])
    assert np.allclose(pm["B1"] @ pm["R"], pm["R"] @ Lam, atol=1e-6)
    R, ld = bd.R_matrix(torch.tensor(lam, dtype=DT), torch.tensor(mu, dtype=DT),
                        torch.tensor(rho, dtype=DT))
    assert np.allclose(R.numpy(), pm["R"], rtol=1e-15, atol=0)
    assert np.allclose(ld.numpy(), np.diag(Lam))
    B1 = bd.Beff1(torch.tensor(lam, dtype=DT), torch.tensor(mu, dtype=DT), torch.tensor(rho, dtype=DT))
    assert np.allclose(B1.numpy(), pm["B1"], rtol=1e-15, atol=0)


def test_rotation_matrix():
    n = torch.tensor([[0.48, -0.6, 0.64]], dtype=DT)
    s, t = bd.tangents(n)
    assert abs(float((n * s).sum())) < 1e-15 and abs(float((n * t).sum())) < 1e-15
    T = bd.T_matrix(n, s, t)[0]
    pm = printed_matrices(_frame_names(n[0].tolist(), s[0].tolist(), t[0].tolist()), which=("T",))
    assert np.allclose(T.numpy(), pm["T"], rtol=1e-15, atol=1e-15)
    # rotating the face-frame strain with the 3x3 frame R = [n s t]
    rng = np.random.default_rng(0)
    e = rng.standard_normal(6)
    ep = np.array([[e[0], e[3], e[5]], [e[3], e[1], e[4]], [e[5], e[4], e[2]]])
    Rf = np.stack([n[0].numpy(), s[0].numpy(), t[0].numpy()], 1)
    eg = Rf @ ep @ Rf.T
    u = np.zeros(10)
    u[:6] = e
    got = T.numpy() @ u
    assert np.allclose(got[:6], [eg[0, 0], eg[1, 1], eg[2, 2], eg[0, 1], eg[1, 2], eg[2, 0]])


def _mat():
    return {k: torch.tensor(v, dtype=DT) for k, v in
            dict(rho=2700.0, lambda0=3.24e10, mu0=3.24e10, gamma_r=37e9, xi0=-0.75, Cd=0.0).items()}


def test_free_surface():
    m = _mat()
    rng = np.random.default_rng(1)
    n = torch.tensor(rng.standard_normal((6, 3)), dtype=DT)
    n = n / torch.linalg.norm(n, dim=1, keepdim=True)
    u = torch.tensor(rng.standard_normal((6, 10)) * 1e-5, dtype=DT)
    u[:, 6:9] *= 1e3
    u[:, 9] = torch.tensor(rng.random(6) * 0.4)
    F = bd.free_surface_flux(u, n, m, AM)
    # rebuild u^b in the face frame and check traction
    lam, mu = bd.effective_lame(u, m, AM)
    s, t = bd.tangents(n)
    T = bd.T_matrix(n, s, t)
    up = torch.linalg.solve(T, u[..., None])[..., 0]
    cp = torch.sqrt((lam + 2 * mu) / m["rho"])
    cs = torch.sqrt(mu / m["rho"])
    sig_nn = (lam + 2 * mu) * up[:, 0] + lam * (up[:, 1] + up[:, 2])
    w1 = -sig_nn / (lam + 2 * mu)
    w2 = -2 * up[:, 3]
    w3 = -2 * up[:, 5]
    vb = torch.stack([up[:, 6] + w1 * cp, up[:, 7] + w2 * cs, up[:, 8] + w3 * cs], 1)
    # closed form: strain flux -sym(v_b (x) n) (global), velocity flux 0
    vg = vb[:, 0:1] * n + vb[:, 1:2] * s + vb[:, 2:3] * t
    E = -0.5 * (vg[:, :, None] * n[:, None, :] + n[:, :, None] * vg[:, None, :])
    want = torch.stack([E[:, 0, 0], E[:, 1, 1], E[:, 2, 2], E[:, 0, 1], E[:, 1, 2], E[:, 2, 0]], 1)
    assert torch.allclose(F[:, :6], want, rtol=1e-12, atol=1e-20)
    assert torch.allclose(F[:, 6:], torch.zeros_like(F[:, 6:]), atol=1e-9)


def test_absorbing_characteristics():
    m = _mat()
    n = torch.tensor([[0.0, 0.6, 0.8]], dtype=DT)
    s, t = bd.tangents(n)
    T = bd.T_matrix(n, s, t)[0]
    lam = m["lambda0"]
    mu = m["mu0"]
    R, ld = bd.R_matrix(lam, mu, m["rho"])
    B1 = bd.Beff1(lam, mu, m["rho"])
    for k in range(10):
        u = (T @ R[:, k])[None] * 1e-6
        F = bd.absorbing_flux(u, n, m, AM)[0]
        if ld[k] > 0:      # outgoing: full normal flux T B1 T^-1 u
            want = T @ (B1 @ R[:, k]) * 1e-6
        else:              # incoming or standing: no flux
            want = torch.zeros(10, dtype=DT)
        assert torch.allclose(F, want, atol=1e-9 * (1e-6 * 6000))
