"""Pins of the oracle's gradients (reverse-mode AD of the oracle step).

* the symmetric form of the Lax-Friedrichs speed used for differentiation
  equals the largest eigenvalue of the 10x10 normal Jacobian (Eq. rusanov-flux)
  taken by the general eigen-solver;
* directional derivatives of one step and of a seismogram misfit, with
  respect to the state, mu0 and C_d, equal central finite differences of the
  forward oracle (independent of automatic differentiation).
"""
import numpy as np
import torch

from oracle import cdm
from oracle.adjoint import diff_from_workload, llf_speed_sym, misfit_gradient, step_vjp
from workloads import make_workload

DT = torch.float64


def _material(n, seed):
    g = torch.Generator().manual_seed(seed)
    mu = 3e10 * (1 + 0.2 * torch.rand(n, generator=g, dtype=DT))
    return dict(rho=2700 * (1 + 0.1 * torch.rand(n, generator=g, dtype=DT)),
                lambda0=3e10 * (1 + 0.2 * torch.rand(n, generator=g, dtype=DT)),
                mu0=mu, gamma_r=37.0 / 32.0 * mu, xi0=torch.full((n,), -0.75, dtype=DT),
                Cd=torch.full((n,), 1e-3, dtype=DT))


def test_llf_speed_symmetric_form_equals_eigenvalue():
    n = 400
    g = torch.Generator().manual_seed(1)
    u = torch.randn(n, 10, generator=g, dtype=DT) * 1e-4
    u[:, 9] = 0.6 * torch.rand(n, generator=g, dtype=DT)       # alpha up to beyond alpha_max
    u[:7, :6] = 0.0                                              # undeformed points (guard)
    nrm = torch.randn(n, 3, generator=g, dtype=DT)
    nrm = nrm / nrm.norm(dim=1, keepdim=True)
    mat = _material(n, 2)
    a = cdm.llf_speed(u, nrm, mat, 0.5)
    b = llf_speed_sym(u, nrm, mat, 0.5)
    assert torch.all(a > 0)
    assert float(((a - b).abs() / a).max()) < 1e-12


def _direction(shape, seed):
    return torch.randn(shape, dtype=DT, generator=torch.Generator().manual_seed(seed))


def _smooth_state(S, w, seed):
    """Projected initial condition plus a random background strain and
    velocity on every mode: no point sits at zero strain, where the law's
    sqrt(I2) term has a cone point and finite differences see no derivative."""
    U = S.project(w.ic).detach()
    bg = _direction(U.shape, seed)
    bg[..., :6] *= 1e-5
    bg[..., 6:9] *= 1e-3
    bg[..., 9] = 0.0
    with torch.no_grad():
        return S.step(U + bg)


def test_step_gradient_matches_central_differences():
    w = make_workload("c2", n=3, N=1)
    S = diff_from_workload(w)
    U = _smooth_state(S, w, 12)
    lam = _direction(U.shape, 3)
    gU, gmu, gcd = step_vjp(S, U, lam)

    def J(U_, mu=None, cd=None):
        saved = S.mat["mu0"], S.mat["Cd"]
        if mu is not None:
            S.mat["mu0"] = mu
        if cd is not None:
            S.mat["Cd"] = cd
        try:
            with torch.no_grad():
                return float((S.step(U_) * lam).sum())
        finally:
            S.mat["mu0"], S.mat["Cd"] = saved

    # state direction
    dU = _direction(U.shape, 4) * U.abs().mean(dim=(0, 1), keepdim=True)
    h = 1e-5
    fd = (J(U + h * dU) - J(U - h * dU)) / (2 * h)
    an = float((gU * dU).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)
    # mu0 and C_d directions
    mu0 = S.mat["mu0"].detach()
    dmu = _direction(mu0.shape, 5) * mu0
    fd = (J(U, mu=mu0 + h * dmu) - J(U, mu=mu0 - h * dmu)) / (2 * h)
    an = float((gmu * dmu).sum())
    assert an != 0.0 and abs(fd - an) <= 1e-6 * abs(an)
    cd0 = S.mat["Cd"].detach()
    dcd = _direction(cd0.shape, 6) * cd0
    fd = (J(U, cd=cd0 + h * dcd) - J(U, cd=cd0 - h * dcd)) / (2 * h)
    an = float((gcd * dcd).sum())
    assert an != 0.0 and abs(fd - an) <= 1e-6 * abs(an)


def test_misfit_gradient_matches_central_differences():
    w = make_workload("c2", n=3, N=1)
    S = diff_from_workload(w)
    U0 = _smooth_state(S, w, 13)
    m = w.mesh
    rec = m["xyz"][m["tets"][[3, 50, 100]]].mean(axis=1)
    nsteps = 3
    dl = _direction((nsteps, 3, 3), 8)
    gmu, gcd, gu0, _ = misfit_gradient(S, U0, nsteps, dl, receivers=rec)
    from oracle.adjoint import seismograms

    def J(mu):
        saved = S.mat["mu0"]
        S.mat["mu0"] = mu
        try:
            with torch.no_grad():
                return float((seismograms(S, U0, nsteps, receivers=rec) * dl).sum())
        finally:
            S.mat["mu0"] = saved

    mu0 = S.mat["mu0"].detach()
    dmu = _direction(mu0.shape, 9) * mu0
    h = 1e-5
    fd = (J(mu0 + h * dmu) - J(mu0 - h * dmu)) / (2 * h)
    an = float((gmu * dmu).sum())
    assert an != 0.0 and abs(fd - an) <= 1e-6 * abs(an)
    assert np.isfinite(gu0.numpy()).all() and np.isfinite(gcd.numpy()).all()
