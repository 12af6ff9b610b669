"""Pins of the oracle's IVM law (Eq. ivm-model, Murnaghan terms off) and of
the step with it.

* the stress is the strain derivative of W = (1 - alpha)(lambda0 I1^2 / 2 +
  mu0 I2) (central differences);
* the Lax-Friedrichs constant from the general eigen-solver of B_n equals the
  damaged P-wave speed sqrt((1 - alpha)(lambda0 + 2 mu0) / rho);
* a periodic uniform state keeps its strain and velocity, and its damage
  follows the ODE dalpha/dt = r_alpha to third order in dt per step (scipy's
  ODE solver gives the exact solution);
* with a negligible damage rate and alpha = 0 the IVM step equals the CDM
  step with no damage (the two laws share only the Hooke limit);
* the boundary fluxes at damage alpha equal the CDM ones of an undamaged
  material with the damaged Lame parameters.
"""
import math

import numpy as np
import torch
from scipy.integrate import solve_ivp

from oracle import cdm, ivm
from oracle.step import OracleSolver
from workloads import make_workload

DT = torch.float64


def _mat(n, seed):
    g = torch.Generator().manual_seed(seed)
    return dict(rho=2700 * (1 + 0.1 * torch.rand(n, generator=g, dtype=DT)),
                lambda0=3e10 * (1 + 0.2 * torch.rand(n, generator=g, dtype=DT)),
                mu0=3e10 * (1 + 0.2 * torch.rand(n, generator=g, dtype=DT)),
                gamma_b=356e3 * (1 + torch.rand(n, generator=g, dtype=DT)),
                tau_b=torch.full((n,), 1e-4, dtype=DT))


def test_stress_is_energy_derivative():
    n = 50
    g = torch.Generator().manual_seed(3)
    u = torch.randn(n, 10, generator=g, dtype=DT) * 1e-4
    u[:, 9] = 0.4 * torch.rand(n, generator=g, dtype=DT)
    mat = _mat(n, 4)

    def W(e):
        I1 = e[:, 0] + e[:, 1] + e[:, 2]
        I2 = (e[:, :3] ** 2).sum(1) + 2 * (e[:, 3:6] ** 2).sum(1)
        return (1 - u[:, 9]) * (0.5 * mat["lambda0"] * I1 ** 2 + mat["mu0"] * I2)

    sig = ivm.stress(u, mat, 0.5)
    h = 1e-9
    for k in range(6):
        ep, em = u[:, :6].clone(), u[:, :6].clone()
        ep[:, k] += h
        em[:, k] -= h
        d = (W(ep) - W(em)) / (2 * h)
        # a shear component appears twice in I2: dW/d eps_k = 2 sigma_k there
        want = d if k < 3 else 0.5 * d
        assert torch.allclose(sig[:, k], want, rtol=1e-6, atol=1e-3)


def test_llf_speed_is_damaged_p_speed():
    n = 40
    g = torch.Generator().manual_seed(5)
    u = torch.randn(n, 10, generator=g, dtype=DT) * 1e-4
    u[:, 9] = 0.7 * torch.rand(n, generator=g, dtype=DT)           # beyond alpha_max too
    nrm = torch.randn(n, 3, generator=g, dtype=DT)
    nrm = nrm / nrm.norm(dim=1, keepdim=True)
    mat = _mat(n, 6)
    ac = torch.clamp(u[:, 9], 0.0, 0.5)
    want = torch.sqrt((1 - ac) * (mat["lambda0"] + 2 * mat["mu0"]) / mat["rho"])
    got = ivm.llf_speed(u, nrm, mat, 0.5)
    assert float(((got - want).abs() / want).max()) < 1e-12


def _uniform(w, eps, alpha0):
    S = OracleSolver(w.mesh["xyz"], w.mesh["tets"], w.mesh["face_tag"], w.mesh["periodic_map"],
                     w.material, w.N, w.dt, alpha_max=w.alpha_max, law=ivm)
    U = torch.zeros(S.E, S.ref.L, 10, dtype=DT)
    c0 = 1.0 / float(S.ref.V[0, 0])                   # constant mode of a unit function
    U[:, 0, :6] = c0 * torch.as_tensor(eps, dtype=DT)
    U[:, 0, 9] = c0 * alpha0
    return S, U, c0


def test_uniform_state_damage_ode_third_order():
    w = make_workload("c1", n=3, N=2, rheology="ivm")
    eps = np.array([2e-4, -1e-4, 0.5e-4, 0.3e-4, -0.2e-4, 0.1e-4])
    alpha0 = 0.05
    lam, mu, gb, tb = (float(w.material[k][0]) for k in ("lambda0", "mu0", "gamma_b", "tau_b"))
    I1 = eps[:3].sum()
    I2 = (eps[:3] ** 2).sum() + 2 * (eps[3:] ** 2).sum()
    e = 0.5 * lam * I1 ** 2 + mu * I2

    def rhs(t, a):
        return [(e - gb * (a[0] / (1 - a[0])) ** 2) / (gb * tb)]

    errs = []
    for dt in (2e-6, 1e-6):
        w.dt = dt
        S, U, c0 = _uniform(w, eps, alpha0)
        U1 = S.step(U)
        # strain and velocity untouched, every element alike
        assert torch.allclose(U1[..., :9], U[..., :9], rtol=0, atol=1e-18)
        a1 = U1[:, 0, 9] / c0
        assert float((a1 - a1[0]).abs().max()) < 1e-15
        exact = solve_ivp(rhs, (0.0, dt), [alpha0], rtol=1e-13, atol=1e-16).y[0, -1]
        assert abs(float(a1[0]) - alpha0) > 1e-4 * alpha0          # damage did move
        errs.append(abs(float(a1[0]) - exact))
    # local error O(dt^3): halving dt divides it by about 8
    assert 5.0 < errs[0] / errs[1] < 11.0, errs


def test_inert_ivm_step_equals_undamaged_cdm_step():
    wi = make_workload("c2", n=2, N=2, rheology="ivm")
    wc = make_workload("c2", n=2, N=2)
    wi.material["gamma_b"] = np.full_like(wi.material["gamma_b"], 1e30)
    wi.material["tau_b"] = np.full_like(wi.material["tau_b"], 1e30)
    wc.material["Cd"] = np.zeros_like(wc.material["Cd"])
    Si = OracleSolver(wi.mesh["xyz"], wi.mesh["tets"], wi.mesh["face_tag"], None,
                      wi.material, wi.N, wi.dt, law=ivm)
    Sc = OracleSolver(wc.mesh["xyz"], wc.mesh["tets"], wc.mesh["face_tag"], None,
                      wc.material, wc.N, wc.dt, law=cdm)
    U = Sc.project(wc.ic)
    U[..., 9] = 0.0
    a, b = Si.step(U), Sc.step(U)
    assert float((a - b).abs().max()) <= 1e-12 * float(b[..., :9].abs().max())


def test_ivm_workload_parameters():
    """Table 2's storage-energy scales on the two kinds of unit, the shortened
    time scale, the elastic model kept; an unknown rheology is refused."""
    wc = make_workload("c2", n=3, N=1)
    wi = make_workload("c2", n=3, N=1, rheology="ivm")
    assert wi.rheology == "ivm" and wc.rheology == "cdm"
    for k in ("rho", "lambda0", "mu0"):
        assert np.array_equal(wi.material[k], wc.material[k])
    cs = np.sqrt(wi.material["mu0"] / wi.material["rho"])
    assert set(np.unique(wi.material["gamma_b"][cs < 1000.0])) == {0.5e3}
    assert set(np.unique(wi.material["gamma_b"][cs >= 1000.0])) == {356e3}
    assert np.all(wi.material["tau_b"] == 1e-4)
    assert wi.dt == wc.dt
    import pytest
    with pytest.raises(ValueError):
        make_workload("c2", n=3, N=1, rheology="plastic")


def test_ivm_boundary_fluxes_are_elastic_with_damaged_moduli():
    """Free-surface and absorbing fluxes under the IVM law at damage alpha
    equal those of an undamaged CDM material with Lame parameters
    (1 - alpha) lambda0, (1 - alpha) mu0 (Eq. effective-ivm): two independent
    routes to the effective moduli."""
    from oracle import boundary
    n = 30
    g = torch.Generator().manual_seed(11)
    u = torch.randn(n, 10, generator=g, dtype=DT) * 1e-4
    u[:, 9] = 0.45 * torch.rand(n, generator=g, dtype=DT)
    nrm = torch.randn(n, 3, generator=g, dtype=DT)
    nrm = nrm / nrm.norm(dim=1, keepdim=True)
    mi = _mat(n, 12)
    gdam = 1.0 - u[:, 9]
    mc = dict(rho=mi["rho"], lambda0=gdam * mi["lambda0"], mu0=gdam * mi["mu0"],
              gamma_r=torch.zeros(n, dtype=DT), xi0=torch.full((n,), -0.75, dtype=DT),
              Cd=torch.zeros(n, dtype=DT))
    u0 = u.clone()
    u0[:, 9] = 0.0
    for fn in (boundary.free_surface_flux, boundary.absorbing_flux):
        a = fn(u, nrm, mi, 0.5, lame=ivm.effective_lame)
        b = fn(u0, nrm, mc, 0.5)
        assert float((a[:, :9] - b[:, :9]).abs().max()) <= 1e-12 * float(b[:, :9].abs().max())
