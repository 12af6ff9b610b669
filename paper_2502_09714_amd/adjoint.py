"""Seismograms as a differentiable function of the per-element shear modulus
mu0 and damage coefficient C_d (torch.autograd), backed by the library's
checkpointed discrete adjoint (dgd_forward_checkpointed / dgd_backward).

    sim = from_workload(w, "fp64")             # mesh, material, sources, receivers
    U0 = sim.get_state()
    mu0 = torch.tensor(w.material["mu0"], requires_grad=True)
    Cd = torch.tensor(w.material["Cd"], requires_grad=True)
    seis = seismograms(sim, mu0, Cd, U0, nsteps=100, every=10)
    loss = 0.5 * ((seis - observed) ** 2).sum()
    loss.backward()                            # mu0.grad, Cd.grad

Marshalling only: the forward steps, the recomputation of each checkpointed
segment and every adjoint kernel run in the HIP library.
"""
import numpy as np
import torch


class _Seismograms(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu0, cd, sim, U0, t0, nsteps, every):
        m = dict(sim.material)
        m["mu0"] = mu0.detach().cpu().numpy().astype(np.float64)
        m["Cd"] = cd.detach().cpu().numpy().astype(np.float64)
        sim.set_material(m["rho"], m["lambda0"], m["mu0"], m["gamma_r"], m["xi0"], m["Cd"])
        sim.set_state(U0)
        sim.set_time(t0)
        sim.clear_seismograms()
        sim.forward_checkpointed(nsteps, every)
        ctx.sim = sim
        ctx.tape = sim.tape_id()
        return torch.as_tensor(sim.get_seismograms(), dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        if ctx.sim.tape_id() != ctx.tape:
            raise RuntimeError("the solver no longer holds the checkpointed run of this graph "
                               "(another forward run or a change of the problem since)")
        gmu, gcd = ctx.sim.backward(g.detach().cpu().numpy())
        return (torch.as_tensor(gmu), torch.as_tensor(gcd), None, None, None, None, None)


def seismograms(sim, mu0, cd, U0, nsteps, every=8, t0=0.0):
    """Receiver velocities (nsteps, nrec, 3) of an nsteps run from U0 (numpy
    (ne, 10, L) or a float64 device tensor) at time t0, with the given mu0 and
    C_d (float64 tensors of shape (ne,)); differentiable in mu0 and C_d."""
    return _Seismograms.apply(mu0, cd, sim, U0, float(t0), int(nsteps), int(every))
