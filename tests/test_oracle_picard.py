"""Pins of the Picard-iteration predictor of the oracle (oracle/picard.py).

* The time-integration matrix integrates polynomials of degree <= N exactly
  (closed form tau^(k+1)/(k+1)).
* Linear limit (alpha = 0, C_d = 0: the CDM law is Hooke's law): the
  converged iteration equals the matrix exponential of the element-local
  operator built from the Cauchy-Kovalevskaya recursion's own ingredients
  (K^e and the flux Jacobians A*_e), scipy's expm, to the collocation error.
* Nonlinear case (damaged rock, alpha = 0.3): the converged iteration equals
  scipy's ODE solver applied to the same local evolution dU/dt = R(U).
* Uniform strain with damage growth: the time points carry the exact linear
  damage growth of the closed-form rate; nothing else moves.
* The full step with this predictor conserves the wave quantities on a
  periodic mesh (the corrector is conservative whatever the predictor).
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
import torch

from oracle.picard import PicardSolver, integration_matrix, local_operator, predict_picard
from oracle.step import OracleSolver
from workloads import make_workload


def _solver(w, cls=OracleSolver, **kw):
    m = w.mesh
    return cls(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"], w.material, w.N, w.dt,
               alpha_max=w.alpha_max, **kw)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_integration_matrix_exact(N):
    from oracle.refmat import RefElement
    tau = RefElement(N).tau.numpy()
    om = integration_matrix(tau).numpy()
    for k in range(N + 1):
        assert np.abs(om @ tau ** k - tau ** (k + 1) / (k + 1)).max() < 1e-14


def _rough_state(S, seed, alpha):
    g = torch.Generator().manual_seed(seed)
    U = torch.randn((S.E, S.ref.L, 10), dtype=torch.float64, generator=g)
    U[..., :6] *= 1e-4
    U[..., 6:9] *= 0.3
    U[..., 9] = 0.0
    U[:, 0, 9] = alpha / float(S.ref.V[0, 0])        # uniform damage alpha
    return U


def _smooth_state(S, seed, alpha):
    """A background strain (far from the cone point of sqrt(I2) at zero strain,
    where the damaged law is not differentiable) with small random mode
    perturbations, uniform damage alpha."""
    g = torch.Generator().manual_seed(seed)
    phi0 = float(S.ref.V[0, 0])
    U = torch.randn((S.E, S.ref.L, 10), dtype=torch.float64, generator=g)
    U[..., :6] *= 1e-5
    U[..., 6:9] *= 0.01
    U[..., 9] = 0.0
    U[:, 0, :6] += torch.tensor([4e-4, -2e-4, 1e-4, 3e-4, -1e-4, 2e-4], dtype=torch.float64) / phi0
    U[:, 0, 9] = alpha / phi0
    return U


def test_linear_limit_matches_matrix_exponential():
    w = make_workload("c1", n=3, N=2)
    S = _solver(w)
    S.dt = w.dt / 8
    U = _rough_state(S, 1, 0.0)
    Uz = predict_picard(S, U, iterations=40)
    # element-local linear operator from the Cauchy-Kovalevskaya ingredients:
    # L(U) = M^-1 (-sum_e K^e U A*_e^T) with A*_e of this (linear) state
    _, Astar = S.predict(U)
    ref = S.ref
    L = ref.L
    for e in (0, 7, 29):
        Lmat = np.zeros((L * 10, L * 10))
        for j in range(L * 10):
            x = torch.zeros((L, 10), dtype=torch.float64)
            x.view(-1)[j] = 1.0
            y = -torch.einsum("ekl,lq,epq->kp", ref.K, x, Astar[e])
            Lmat[:, j] = (ref.Minv @ y).reshape(-1).numpy()
        u0 = U[e].reshape(-1).numpy()
        for z, tz in enumerate(ref.tau.numpy()):
            want = scipy.linalg.expm(tz * S.dt * Lmat) @ u0
            got = Uz[z, e].reshape(-1).numpy()
            assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-11


def test_nonlinear_matches_ode_solver():
    """Converged iteration = Gauss-Legendre collocation solution of the local
    evolution; its time-point values differ from the exact solution (scipy's
    DOP853 at rtol 1e-13) by the collocation error, which falls as dt^(N+1)
    (the stage order): both its size and its rate are checked."""
    w = make_workload("c2", n=1, N=2)
    S = _solver(w)
    U = _smooth_state(S, 2, 0.3)
    shape = U.shape
    errs = []
    for div in (4, 16):
        S.dt = w.dt / div
        Uz = predict_picard(S, U, iterations=40)
        assert float((predict_picard(S, U, iterations=39) - Uz).abs().max()) == 0.0

        def rhs(t, y):
            return local_operator(S, torch.as_tensor(y).reshape(shape)).reshape(-1).numpy()

        tz = S.ref.tau.numpy() * S.dt
        sol = scipy.integrate.solve_ivp(rhs, (0.0, S.dt), U.reshape(-1).numpy(), method="DOP853",
                                        t_eval=tz, rtol=1e-13, atol=1e-20)
        assert sol.success
        u0 = U.reshape(-1).numpy()
        errs.append(max(np.linalg.norm(Uz[z].reshape(-1).numpy() - sol.y[:, z]) /
                        np.linalg.norm(sol.y[:, z] - u0) for z in range(S.ref.Nt)))
    assert errs[1] < 1e-7
    assert errs[0] / errs[1] > 4.0 ** (S.N + 1) / 2


def test_uniform_strain_damage_growth():
    w = make_workload("c1", n=3, N=3)
    w.material["Cd"] = np.full(w.ne, 1e8 / 37e9)
    S = _solver(w)
    eps = np.array([2e-5, -1e-5, 0.5e-5, 3e-5, 0.0, -1e-5])
    U = torch.zeros((S.E, S.ref.L, 10), dtype=torch.float64)
    phi0 = float(S.ref.V[0, 0])
    U[:, 0, :6] = torch.as_tensor(eps) / phi0
    U[:, 0, 9] = 0.1 / phi0
    I1 = eps[:3].sum()
    I2 = (eps[:3] ** 2).sum() + 2 * (eps[3:] ** 2).sum()
    xi = I1 / math.sqrt(I2)
    r = 1e8 / 37e9 * 37e9 * I2 * (xi + 0.75)            # C_d gamma_r I2 (xi - xi0)
    Uz = predict_picard(S, U)
    for z, tz in enumerate(S.ref.tau.numpy()):
        d = (Uz[z] - U).numpy()
        # strain and velocity stay (to rounding against their own scales:
        # |eps| and the particle velocity c_p |eps| it would drive)
        assert np.abs(d[..., :6]).max() < 1e-12 * np.abs(eps).max()
        assert np.abs(d[..., 6:9]).max() < 1e-12 * 6000.0 * np.abs(eps).max()
        assert np.allclose(d[:, 0, 9] * phi0, r * tz * S.dt, rtol=1e-12, atol=0)
        assert np.abs(d[:, 1:, 9]).max() < 1e-13 * abs(r * S.dt)


def test_picard_step_conserves():
    w = make_workload("c2", n=3, N=2, periodic=True)
    S = _solver(w, PicardSolver)
    U = S.project(w.ic)
    phi0 = float(S.ref.V[0, 0])
    vol = S.mesh.detJ
    tot0 = (vol[:, None] * U[:, 0, :9]).sum(0)
    U1 = S.step(U)
    tot1 = (vol[:, None] * U1[:, 0, :9]).sum(0)
    # every wave quantity against its own magnitude on the mesh
    scale = torch.maximum((vol[:, None] * U[:, 0, :9].abs()).sum(0),
                          (vol[:, None] * U1[:, 0, :9].abs()).sum(0))
    assert bool(((tot1 - tot0).abs() <= 1e-12 * scale).all())
    assert float((U1 - U).abs().max()) > 0
