"""One ADER-DG step of the CDM (or IVM) system (oracle), Section 2.2 and Appendix A.

Modal coefficients U[m, l, p] (element m, mode l, quantity p) of the expansion
u^h_p = sum_l U_lp phi_l (Eq. modal dg space).  One global time step
t_n -> t_n + dt (global time stepping):

Prediction (Appendix A.1)
  1. nodal values u_q = sum_l V_ql U_lp at the volume quadrature points;
  2. cell-averaged Jacobians  Bbar^d = int B^d(u) dV / V_e, taken as the
     quadrature average of the pointwise Jacobian (Eq. CKIter text);
  3. Cauchy-Kovalevskaya recursion in the reference element (Eq.
     CKIter-ref-matrix), with A*_e = sum_d Theta^{-1}_ed Bbar^d:
       M D^i = - sum_e K^e D^{i-1} (A*_e)^T            i = 1..N
     plus, for i = 1 only, the damage source int s(u^{t_n}) phi_k evaluated
     on the nodal points (Eq. CKIter-ref-source);
  4. Taylor series U(t_n + tau) = sum_i tau^i / i! D^i (Eq. taylor_expansion),
     truncated at the polynomial degree N.

Correction (Appendix A.2, Eq. time-integrated)
  5. volume term: at every time point tau_z, nodal values -> F^d -> modal
     F^d_l (L2 projection), time-integrated with gamma_z, contracted with the
     stiffness int dphi_k/dx_d phi_l (Eq. 3rd term);
  6. source term: nodal r_alpha -> modal S_l, time-integrated, times the mass
     matrix (Eq. rhs term);
  7. face term: local Lax-Friedrichs flux (Eq. rusanov-flux) at every face
     quadrature point (shared by both sides, see :mod:`oracle.mesh`) and time point, C the largest eigenvalue of B_n at the
     mean state (the larger of the two sides' materials), summed with
     beta_i gamma_z |S_f| dt (Eq. 2nd term); boundary faces use the
     free-surface or absorbing flux of Appendix A.3;
  8. |J| M (U^{n+1} - U^n) = dt (volume + source - face), everything divided by
     |J| so that only reference matrices remain.
"""
import numpy as np
import torch

from . import boundary, cdm
from .mesh import OracleMesh
from .refmat import RefElement

DT = torch.float64
TAG_FREE = 1
TAG_ABSORB = 2


class OracleSolver:
    """Plain FP64 CPU reference solver for one workload."""

    def __init__(self, xyz, tets, face_tag, periodic_map, material, N, dt,
                 alpha_max=0.5, i2_min=cdm.I2_MIN_F64, llf_speed=None, law=cdm):
        self.N = N
        # the rheology's pointwise law: oracle.cdm (Eq. cdb-model) or
        # oracle.ivm (Eq. ivm-model)
        self.law = law
        # largest eigenvalue of B_n (Eq. rusanov-flux); replaceable by an
        # equal, differentiable form (oracle.adjoint)
        self.llf_speed = law.llf_speed if llf_speed is None else llf_speed
        self.ref = RefElement(N)
        self.mesh = OracleMesh(xyz, tets, face_tag, periodic_map, self.ref)
        self.E = self.mesh.E
        self.mat = {k: torch.as_tensor(np.asarray(material[k], dtype=np.float64))
                    for k in law.MAT_KEYS}
        self.dt = float(dt)
        self.alpha_max = float(alpha_max)
        self.i2_min = float(i2_min)

    # -- helpers --------------------------------------------------------------
    def _mat(self, idx=None, extra_dims=0):
        out = {}
        for k, v in self.mat.items():
            t = v if idx is None else v[idx]
            out[k] = t.reshape(t.shape + (1,) * extra_dims)
        return out

    def quadrature_points(self):
        """Physical coordinates of the volume quadrature points (E, Q, 3)."""
        m = self.mesh
        return m.X0[:, None, :] + torch.einsum("mde,qe->mqd", m.J, self.ref.xq)

    def project(self, ic):
        """L2 projection of ic(x, elem) -> U (E, L, 10)."""
        x = self.quadrature_points()
        E, Q = x.shape[:2]
        elem = np.repeat(np.arange(E), Q)
        vals = torch.as_tensor(ic(x.reshape(-1, 3).numpy(), elem), dtype=DT)
        return torch.einsum("lq,mqp->mlp", self.ref.P, vals.reshape(E, Q, 10))

    # -- prediction -------------------------------------------------------------
    def predict(self, U):
        ref, m = self.ref, self.mesh
        am, i2 = self.alpha_max, self.i2_min
        mat_q = self._mat(extra_dims=1)
        uq = torch.einsum("ql,mlp->mqp", ref.V, U)
        B = self.law.flux_jacobian(uq, mat_q, am, i2)                 # (E,Q,3,10,10)
        Bbar = torch.einsum("q,mqdij->mdij", ref.wq, B) / ref.wq.sum()
        Astar = torch.einsum("med,mdij->meij", m.Jinv, Bbar)           # (E,3,10,10)
        D = [U]
        for i in range(1, self.N + 1):
            rhs = -torch.einsum("ekl,mlq,mepq->mkp", ref.K, D[i - 1], Astar)
            if i == 1:
                r = self.law.r_alpha(uq, mat_q, am, i2)               # (E,Q)
                src = torch.einsum("ql,q,mq->ml", ref.V, ref.wq, r)
                rhs = rhs.clone()
                rhs[..., 9] = rhs[..., 9] + src
            D.append(torch.einsum("kl,mlp->mkp", ref.Minv, rhs))
        return D, Astar

    def time_points(self, D):
        """U(t_n + tau_z dt) for every Gauss time point, (Nt, E, L, 10)."""
        out = []
        for tz in self.ref.tau:
            h = float(tz) * self.dt
            acc = torch.zeros_like(D[0])
            fac = 1.0
            for i, Di in enumerate(D):
                if i > 0:
                    fac = fac * h / i
                acc = acc + fac * Di
            out.append(acc)
        return torch.stack(out)

    # -- correction ---------------------------------------------------------------
    def volume_and_source(self, Uz):
        ref, m = self.ref, self.mesh
        am, i2 = self.alpha_max, self.i2_min
        mat_q = self._mat(extra_dims=1)
        Fint = 0.0
        Sint = 0.0
        for z in range(ref.Nt):
            u = torch.einsum("ql,mlp->mqp", ref.V, Uz[z])
            F = self.law.flux(u, mat_q, am, i2)                       # (E,Q,3,10)
            Fmod = torch.einsum("lq,mqdp->mdlp", ref.P, F)            # modal flux
            S = self.law.r_alpha(u, mat_q, am, i2)
            Smod = torch.einsum("lq,mq->ml", ref.P, S)
            Fint = Fint + ref.gamma[z] * Fmod
            Sint = Sint + ref.gamma[z] * Smod
        # int dphi_k/dx_d phi_l = sum_e Theta^{-1}_ed int dphi_k/dxi_e phi_l
        vol = self.dt * torch.einsum("med,ekl,mdlp->mkp", m.Jinv, ref.Kstiff, Fint)
        src = torch.zeros_like(vol)
        src[..., 9] = self.dt * torch.einsum("kl,ml->mk", ref.M, Sint)
        return vol, src

    def face_fluxes(self, Uz):
        """Time-integrated numerical flux at every face point: (E, 4, Ns, 10)."""
        ref, m = self.ref, self.mesh
        am, i2 = self.alpha_max, self.i2_min
        E = self.E
        out = torch.zeros((E, 4, ref.Ns, 10), dtype=DT)
        for f in range(4):
            inter = np.nonzero(m.nbr[:, f] >= 0)[0]
            free = np.nonzero(m.face_tag[:, f] == TAG_FREE)[0]
            absb = np.nonzero(m.face_tag[:, f] == TAG_ABSORB)[0]
            if inter.size:
                me = torch.as_tensor(inter)
                nb = torch.as_tensor(m.nbr[inter, f])
                n = m.normal[me, f][:, None, :].expand(len(inter), ref.Ns, 3)
                mat_m = self._mat(me, extra_dims=1)
                mat_p = self._mat(nb, extra_dims=1)
                acc = 0.0
                for z in range(ref.Nt):
                    uM = torch.einsum("mil,mlp->mip", m.Fface[me, f], Uz[z][me])
                    uP = torch.einsum("mil,mlp->mip", m.Fnbr[me, f], Uz[z][nb])
                    FM = torch.einsum("mid,midp->mip", n, self.law.flux(uM, mat_m, am, i2))
                    FP = torch.einsum("mid,midp->mip", n, self.law.flux(uP, mat_p, am, i2))
                    ubar = 0.5 * (uM + uP)
                    C = torch.maximum(self.llf_speed(ubar, n, mat_m, am, i2),
                                      self.llf_speed(ubar, n, mat_p, am, i2))
                    Fs = 0.5 * (FM + FP) + 0.5 * C[..., None] * (uM - uP)
                    acc = acc + ref.gamma[z] * Fs
                out[me, f] = acc
            for idx, fn in ((free, boundary.free_surface_flux),
                            (absb, boundary.absorbing_flux)):
                if not idx.size:
                    continue
                me = torch.as_tensor(idx)
                n = m.normal[me, f][:, None, :].expand(len(idx), ref.Ns, 3)
                mat_m = self._mat(me, extra_dims=1)
                acc = 0.0
                for z in range(ref.Nt):
                    uM = torch.einsum("mil,mlp->mip", m.Fface[me, f], Uz[z][me])
                    # effective Lame parameters: the law's own (IVM) or the
                    # CDM ones of oracle.boundary
                    acc = acc + ref.gamma[z] * fn(uM, n, mat_m, am, i2,
                                                  lame=getattr(self.law, "effective_lame", None))
                out[me, f] = acc
        return out

    def face_term(self, Uz):
        ref, m = self.ref, self.mesh
        Fint = self.face_fluxes(Uz)
        scale = self.dt * m.area / m.detJ[:, None]                    # (E, 4)
        # lift: beta_i phi_k(x_i) at the element's own view of the face points
        return torch.einsum("mf,i,mfik,mfip->mkp", scale, ref.beta, m.Fface, Fint)

    def step(self, U):
        D, _ = self.predict(U)
        Uz = self.time_points(D)
        vol, src = self.volume_and_source(Uz)
        face = self.face_term(Uz)
        rhs = vol + src - face
        return U + torch.einsum("kl,mlp->mkp", self.ref.Minv, rhs)

    def run(self, U, nsteps, callback=None):
        for n in range(nsteps):
            U = self.step(U)
            if callback is not None:
                callback(n, U)
        return U


def from_workload(w, **kw):
    """OracleSolver for a :class:`workloads.Workload` (its rheology's law)."""
    from . import ivm
    m = w.mesh
    kw.setdefault("law", ivm if getattr(w, "rheology", "cdm") == "ivm" else cdm)
    return OracleSolver(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"],
                        w.material, w.N, w.dt, alpha_max=w.alpha_max, **kw)
