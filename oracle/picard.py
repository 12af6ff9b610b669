"""Picard-iteration predictor (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Discussion (Section 5.1) names a discrete Picard iteration as the
replacement for the linearised Cauchy-Kovalevskaya procedure of the prediction
step (Appendix A.1, Eqs. CKIter, CKIter-ref-matrix), to keep high-order
accuracy for nonlinear rheologies; it gives no formulas.  Reading used here:

* The prediction over [t_n, t_n + dt] solves the element-local evolution that
  the Cauchy-Kovalevskaya recursion differentiates, in strong form and without
  linearising it:
      dU/dt = R(U) = M^-1 [ - sum_e sum_d Theta^-1_ed K^e Fhat^d(U) + s(U) ],
  with Fhat^d(U) = P F^d(V U) the L2 projection of the pointwise flux of Eq.
  nonlinear hyper pdes (nodal evaluation and projection as in Eq. 3rd term)
  and s(U) the projected damage source in the alpha row.  At a linear flux
  F^d(u) = B^d u this R is the right-hand side of the first Cauchy-Kovalevskaya
  derivative, D^1 = R(U^n).
* U(t_n + tau dt) is the polynomial of degree N in time through its values U_z
  at the Gauss-Legendre points tau_z used by the corrector (Eq. 2nd term, 3rd
  term), and the collocation equations
      U_z = U^n + dt sum_z' Omega_zz' R(U_z'),   Omega_zz' = int_0^tau_z l_z'(s) ds
  (l_z' the Lagrange polynomials of the points) are solved by Picard
  iteration from U_z = U^n; every iteration gains one order in dt, and the
  number of iterations is N + 1 unless stated.
* The corrector (volume and source terms, faces, update) uses these U_z in
  place of the Taylor sums of Eq. taylor_expansion.
"""
import numpy as np
import torch

from .step import OracleSolver

DT = torch.float64


def integration_matrix(tau):
    """Omega[z, z'] = int_0^{tau_z} l_z'(s) ds for the Lagrange polynomials
    l_z' of the points tau (numpy polynomial arithmetic, float64)."""
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    om = np.zeros((n, n))
    for j in range(n):
        c = np.array([1.0])
        for k in range(n):
            if k != j:
                c = np.polynomial.polynomial.polymul(c, np.array([-tau[k], 1.0]) / (tau[j] - tau[k]))
        ci = np.polynomial.polynomial.polyint(c)
        om[:, j] = np.polynomial.polynomial.polyval(tau, ci)
    return torch.as_tensor(om, dtype=DT)


def local_operator(S, U):
    """R(U) of the element-local strong-form evolution, U (E, L, 10)."""
    ref, m = S.ref, S.mesh
    am, i2 = S.alpha_max, S.i2_min
    mat_q = S._mat(extra_dims=1)
    uq = torch.einsum("ql,mlp->mqp", ref.V, U)
    F = S.law.flux(uq, mat_q, am, i2)                                 # (E, Q, 3, 10)
    Fhat = torch.einsum("lq,mqdp->mdlp", ref.P, F)                    # (E, 3, L, 10)
    div = torch.einsum("med,ekl,mdlp->mkp", m.Jinv, ref.K, Fhat)
    r = S.law.r_alpha(uq, mat_q, am, i2)                              # (E, Q)
    src = torch.einsum("ql,q,mq->ml", ref.V, ref.wq, r)
    rhs = -div
    rhs = rhs.clone()
    rhs[..., 9] = rhs[..., 9] + src
    return torch.einsum("kl,mlp->mkp", ref.Minv, rhs)


def predict_picard(S, U, iterations=None):
    """Time-point states (Nt, E, L, 10) after `iterations` Picard sweeps of
    the collocation equations (default N + 1)."""
    K = S.N + 1 if iterations is None else int(iterations)
    om = integration_matrix(S.ref.tau.numpy())
    Nt = S.ref.Nt
    Uz = [U for _ in range(Nt)]
    for _ in range(K):
        R = [local_operator(S, Uz[z]) for z in range(Nt)]
        Uz = [U + S.dt * sum(om[z, j] * R[j] for j in range(Nt)) for z in range(Nt)]
    return torch.stack(Uz)


class PicardSolver(OracleSolver):
    """OracleSolver whose predictor is the Picard iteration above."""

    def __init__(self, *a, iterations=None, **kw):
        super().__init__(*a, **kw)
        self.iterations = self.N + 1 if iterations is None else int(iterations)

    def step(self, U):
        Uz = predict_picard(self, U, self.iterations)
        vol, src = self.volume_and_source(Uz)
        face = self.face_term(Uz)
        return U + torch.einsum("kl,mlp->mkp", self.ref.Minv, vol + src - face)


def picard_from_workload(w, iterations=None, **kw):
    from . import cdm, ivm
    m = w.mesh
    kw.setdefault("law", ivm if getattr(w, "rheology", "cdm") == "ivm" else cdm)
    return PicardSolver(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"], w.material,
                        w.N, w.dt, alpha_max=w.alpha_max, iterations=iterations, **kw)
