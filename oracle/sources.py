"""Point moment-tensor sources and receivers (oracle).

The paper drives its regional run with a kinematic finite-fault source and
records velocity seismograms at stations (Section 4); neither formula is
printed for this setting.  Readings used here:

* a point source with moment tensor M_ij(t) = M6_ij S(t - t_onset) acts as
  the body force f_i = -d_j (M_ij(t) delta(x - x_s)) in the momentum
  equation, so that int_T phi_k f_i dV = M_ij dphi_k/dx_j(x_s).  Its exact
  integral over one step is added to the velocity modes of the element that
  contains x_s after the DG update:
      M dU_k,v_i = M6_ij dphi_k/dx_j(x_s) [G(t_{n+1}) - G(t_n)] / (rho |J|)
  with G the antiderivative of the moment function S (S itself being the
  antiderivative of the moment-rate wavelet):
      Ricker moment rate (1 - 2 a tau^2) e^{-a tau^2}, a = (pi f0)^2:
          S = tau e^{-a tau^2},  G = -e^{-a tau^2} / (2a)
      Gaussian moment rate e^{-tau^2/w^2} / (w sqrt(pi)):
          S = (1 + erf(tau/w))/2,  G = (tau (1 + erf(tau/w)) + w e^{-tau^2/w^2}/sqrt(pi))/2
* a receiver records (v_x, v_y, v_z) = sum_l U_l,v phi_l(xi_r) at the end of
  every step.
* a point belongs to the lowest-numbered element whose closed tetrahedron
  contains it (barycentric coordinates >= -1e-12).
"""
import math

import numpy as np
import torch

DT = torch.float64
STF_RICKER = 0
STF_GAUSSIAN = 1


def locate(mesh, pts, tol=1e-12):
    """Element index and reference coordinates of every point."""
    pts = torch.as_tensor(np.asarray(pts, dtype=np.float64))
    elems, xis = [], []
    for p in pts:
        xi = torch.einsum("med,md->me", mesh.Jinv, p[None, :] - mesh.X0)   # (E,3)
        bary = torch.cat([1.0 - xi.sum(1, keepdim=True), xi], 1)
        inside = torch.nonzero((bary >= -tol).all(1))
        if inside.numel() == 0:
            raise ValueError("point outside the mesh")
        m = int(inside[0, 0])
        elems.append(m)
        xis.append(xi[m])
    return np.asarray(elems, dtype=np.int64), torch.stack(xis)


def stf_antiderivative2(kind, tau, param):
    """G(tau): second antiderivative of the moment-rate wavelet."""
    if kind == STF_RICKER:
        a = (math.pi * param) ** 2
        return -math.exp(-a * tau * tau) / (2.0 * a)
    w = param
    return 0.5 * (tau * (1.0 + math.erf(tau / w))
                  + w * math.exp(-tau * tau / (w * w)) / math.sqrt(math.pi))


class PointSources:
    def __init__(self, solver, xyz, M6, t_onset, stf_param, stf_kind):
        self.solver = solver
        self.elem, self.xi = locate(solver.mesh, xyz)
        self.M6 = np.asarray(M6, dtype=np.float64)
        self.t_onset = np.asarray(t_onset, dtype=np.float64)
        self.param = np.asarray(stf_param, dtype=np.float64)
        self.kind = int(stf_kind)
        m = solver.mesh
        g = solver.ref.basis.gradients(self.xi)                 # (n, 3, L) d/dxi_e
        Jinv = m.Jinv[torch.as_tensor(self.elem)]               # (n, e, d)
        self.dphi = torch.einsum("nel,ned->ndl", g, Jinv)        # d phi / dx_d

    def increment(self, t0, t1):
        """dU (E, L, 10) contributed over [t0, t1]."""
        s = self.solver
        dU = torch.zeros((s.E, s.ref.L, 10), dtype=DT)
        sym = ((0, 3, 5), (3, 1, 4), (5, 4, 2))
        for k in range(len(self.elem)):
            m = int(self.elem[k])
            dG = (stf_antiderivative2(self.kind, t1 - self.t_onset[k], self.param[k])
                  - stf_antiderivative2(self.kind, t0 - self.t_onset[k], self.param[k]))
            fac = dG / (float(s.mat["rho"][m]) * float(s.mesh.detJ[m]))
            for i in range(3):
                rhs = torch.zeros(s.ref.L, dtype=DT)
                for j in range(3):
                    rhs = rhs + self.M6[k, sym[i][j]] * self.dphi[k, j]
                dU[m, :, 6 + i] += fac * (s.ref.Minv @ rhs)
        return dU


class Receivers:
    def __init__(self, solver, xyz):
        self.elem, self.xi = locate(solver.mesh, xyz)
        self.phi = solver.ref.basis.values(self.xi)              # (nrec, L)

    def sample(self, U):
        """(nrec, 3) velocities."""
        return torch.einsum("rl,rlp->rp", self.phi, U[torch.as_tensor(self.elem)][:, :, 6:9])
