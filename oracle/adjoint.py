"""Gradients of the discrete step and of a seismogram misfit (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes forward seismograms; the gradients checked here are those
of the discrete update of :mod:`oracle.step` (Appendix A.1-A.3 with the law of
Eq. cdb-model), taken by reverse-mode automatic differentiation of the oracle
itself with respect to the modal state and the per-element shear modulus mu0
and damage coefficient C_d.  Every derivative is therefore the derivative of
the plain definition; nothing is hand-derived.

One change to the forward oracle is needed for differentiation: the local
Lax-Friedrichs constant.  The forward oracle takes the largest real part of the
eigenvalues of the 10x10 normal Jacobian B_n (Eq. rusanov-flux) from a general
eigen-solver, whose derivative is ill-conditioned at the zero eigenvalue of
multiplicity four.  The eigenvalues of B_n are 0 and +-sqrt of the eigenvalues
of the symmetric 3x3 velocity block of B_n^2 (strain rows feed only from
velocities, velocity rows only from strains and alpha, alpha carries no
flux), so the same number is sqrt(largest eigenvalue of (B_n^2)_vv), taken by a
symmetric eigen-solver.  :class:`DiffSolver` uses that form; the two forms
are pinned equal by a test.

Non-smooth points take PyTorch's conventions: clamp passes the derivative on
the closed interval, ``where`` routes it to the selected branch, and
``maximum`` gives half to each argument at a tie.
"""
import torch

from . import cdm
from .sources import PointSources, Receivers
from .step import OracleSolver

DT = torch.float64


def llf_speed_sym(u, n, mat, alpha_max, i2_min=cdm.I2_MIN_F64):
    """sqrt(lambda_max((B_n^2)_vv)): the largest eigenvalue of B_n (Eq.
    rusanov-flux) through a symmetric 3x3 eigenproblem."""
    Bn = cdm.normal_jacobian(u, n, mat, alpha_max, i2_min)
    Q = Bn[..., 6:9, :] @ Bn[..., :, 6:9]
    Q = 0.5 * (Q + Q.transpose(-1, -2))
    lm = torch.linalg.eigvalsh(Q)[..., -1]
    return torch.sqrt(torch.clamp(lm, min=0.0))


class DiffSolver(OracleSolver):
    """OracleSolver whose mu0 and C_d are leaf tensors and whose LLF constant
    takes the symmetric form above."""

    def __init__(self, *a, **kw):
        kw.setdefault("llf_speed", llf_speed_sym)
        super().__init__(*a, **kw)
        self.mat["mu0"] = self.mat["mu0"].clone().requires_grad_(True)
        self.mat["Cd"] = self.mat["Cd"].clone().requires_grad_(True)

    def zero_grads(self):
        for k in ("mu0", "Cd"):
            self.mat[k].grad = None


def diff_from_workload(w, **kw):
    m = w.mesh
    return DiffSolver(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"],
                      w.material, w.N, w.dt, alpha_max=w.alpha_max, **kw)


def step_vjp(S, U, lam):
    """(lam^T dU^{n+1}/dU^n, lam^T dU^{n+1}/dmu0, lam^T dU^{n+1}/dC_d) for one
    step of the DiffSolver S at U (E, L, 10); lam (E, L, 10)."""
    S.zero_grads()
    U = U.detach().clone().requires_grad_(True)
    out = S.step(U)
    (out * lam).sum().backward()
    return U.grad.detach(), S.mat["mu0"].grad.detach().clone(), S.mat["Cd"].grad.detach().clone()


def seismograms(S, U0, nsteps, t0=0.0, sources=None, receivers=None):
    """Seismograms (nsteps, nrec, 3) of a run: step, then the source
    increment over [t, t + dt], then the receivers sample the new state."""
    src = PointSources(S, **sources) if sources is not None else None
    rec = Receivers(S, receivers)
    U = U0
    t = t0
    out = []
    for _ in range(nsteps):
        U = S.step(U)
        if src is not None:
            U = U + src.increment(t, t + S.dt)
        t += S.dt
        out.append(rec.sample(U))
    return torch.stack(out)


def misfit_gradient(S, U0, nsteps, dl_dseis, t0=0.0, sources=None, receivers=None):
    """Gradients of J = sum(dl_dseis * seismograms) (a linearised misfit; any
    misfit's gradient is this with dl_dseis = dJ/dseismograms) with respect to
    mu0, C_d and U0."""
    S.zero_grads()
    U0 = U0.detach().clone().requires_grad_(True)
    seis = seismograms(S, U0, nsteps, t0, sources, receivers)
    (seis * torch.as_tensor(dl_dseis, dtype=DT)).sum().backward()
    return (S.mat["mu0"].grad.detach().clone(), S.mat["Cd"].grad.detach().clone(),
            U0.grad.detach(), seis.detach())
