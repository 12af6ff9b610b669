"""FP64 diagnostics (oracle).

The paper reports maps of co-seismic wave-speed change (Section 4.2) without a
formula; readings used here:

* total energy  E = sum_m |J|_m sum_q w_q [rho |v|^2 / 2 + W(eps, alpha)],
  W = lambda0 I1^2/2 + (mu0 + alpha xi0 gamma_r) I2 - alpha gamma_r I1 sqrt(I2)
  (the strain-energy density whose strain derivative is the CDM stress,
  Eq. cdb-model);
* damage-only shear-wave-speed change of element m:
  dc_s/c_s = sqrt(max(mu0 + abar xi0 gamma_r, 0) / mu0) - 1,
  abar the clamped cell mean of alpha (mu0 + alpha xi0 gamma_r is the
  damaged shear modulus of the stress law); for the IVM law
  dc_s/c_s = sqrt(1 - abar) - 1 (shear modulus (1 - alpha) mu0).
"""
import math

import torch

from . import cdm

DT = torch.float64


def energy(solver, U):
    ref, m = solver.ref, solver.mesh
    u = torch.einsum("ql,mlp->mqp", ref.V, U)
    mat = solver._mat(extra_dims=1)
    kin = 0.5 * mat["rho"] * (u[..., 6:9] ** 2).sum(-1)
    W = cdm.energy_density(u, mat, solver.alpha_max, solver.i2_min)
    return float(torch.einsum("m,q,mq->", m.detJ, ref.wq, kin + W))


def wavespeed_change(solver, U):
    # cell mean of alpha = int alpha / |T| with |T| = 1/6
    phi0_int = float(solver.ref.wq @ solver.ref.V[:, 0])
    abar = 6.0 * phi0_int * U[:, 0, 9]
    abar = torch.clamp(abar, 0.0, solver.alpha_max)
    if solver.law.__name__.endswith("ivm"):
        # shear modulus (1 - alpha) mu0 (Eq. effective-ivm)
        return torch.sqrt(1.0 - abar) - 1.0
    mu0 = solver.mat["mu0"]
    mud = torch.clamp(mu0 + abar * solver.mat["xi0"] * solver.mat["gamma_r"], min=0.0)
    return torch.sqrt(mud / mu0) - 1.0
