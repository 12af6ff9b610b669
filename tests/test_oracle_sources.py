"""Pins of the oracle's point sources, receivers and diagnostics.

* the second antiderivatives of the moment-rate wavelets differentiate back
  to the wavelets (finite differences, twice);
* point location returns an element whose closed tetrahedron holds the point;
* receivers reproduce a field that lies in the approximation space exactly;
* a moment-tensor source exerts no net force (only the velocity modes with a
  non-constant gradient move) and its momentum change is the dipole formula;
* the energy of a plane P wave equals the closed form, and the wave-speed
  change is zero without damage and negative with it.
"""
import math

import numpy as np
import torch

from oracle.diagnostics import energy, wavespeed_change
from oracle.sources import (STF_GAUSSIAN, STF_RICKER, PointSources, Receivers,
                            locate, stf_antiderivative2)
from oracle.step import from_workload
from workloads import make_workload


def _ricker(t, f0):
    a = (math.pi * f0) ** 2
    return (1 - 2 * a * t * t) * math.exp(-a * t * t)


def _gauss(t, w):
    return math.exp(-t * t / (w * w)) / (w * math.sqrt(math.pi))


def test_stf_antiderivatives():
    h = 1e-4
    for kind, p, fn in ((STF_RICKER, 2.0, _ricker), (STF_GAUSSIAN, 0.1, _gauss)):
        for t in np.linspace(-0.4, 0.4, 9):
            G = lambda x: stf_antiderivative2(kind, x, p)
            d2 = (G(t + h) - 2 * G(t) + G(t - h)) / (h * h)
            assert abs(d2 - fn(t, p)) < 1e-5 * (1 + abs(fn(t, p))) * (1 if kind else 10)
        assert abs(stf_antiderivative2(kind, -10.0, p)) < 1e-12


def test_locate_and_receivers():
    w = make_workload("c4", n=4, N=2)
    S = from_workload(w)
    elem, xi = locate(S.mesh, w.receivers)
    for k in range(len(elem)):
        x = S.mesh.X0[elem[k]] + S.mesh.J[elem[k]] @ xi[k]
        assert torch.allclose(x, torch.tensor(w.receivers[k]), atol=1e-9)
        assert (xi[k] >= -1e-12).all() and xi[k].sum() <= 1 + 1e-12
    # linear field v = (x, 2y, -z) is represented exactly for N >= 1
    U = S.project(lambda x, e: np.concatenate([np.zeros((x.shape[0], 6)),
                                               np.stack([x[:, 0], 2 * x[:, 1], -x[:, 2]], 1),
                                               np.zeros((x.shape[0], 1))], 1))
    rec = Receivers(S, w.receivers).sample(U)
    r = torch.tensor(w.receivers)
    assert torch.allclose(rec, torch.stack([r[:, 0], 2 * r[:, 1], -r[:, 2]], 1), rtol=1e-12)


def test_point_source_dipole():
    w = make_workload("c4", n=4, N=2)
    S = from_workload(w)
    src = PointSources(S, **w.sources)
    dU = src.increment(0.4, 0.7)
    m = int(src.elem[0])
    assert torch.count_nonzero(dU[torch.arange(S.E) != m]) == 0
    # no net force: the constant mode of velocity does not move
    assert torch.allclose(dU[m, 0, 6:9], torch.zeros(3, dtype=torch.float64), atol=1e-12 * float(dU.abs().max()))
    # int x_j rho dv_i dV = M_ij dG  (first moment of f = -div(M delta))
    q = S.quadrature_points()[m]
    wq = S.ref.wq * S.mesh.detJ[m]
    v = S.ref.V @ dU[m][:, 6:9]                                  # (Q, 3)
    rho = float(S.mat["rho"][m])
    mom = torch.einsum("q,qj,qi->ij", wq, q, rho * v)
    dG = (stf_antiderivative2(STF_RICKER, 0.7 - 0.6, 2.0)
          - stf_antiderivative2(STF_RICKER, 0.4 - 0.6, 2.0))
    M6 = w.sources["M6"][0]
    M = np.array([[M6[0], M6[3], M6[5]], [M6[3], M6[1], M6[4]], [M6[5], M6[4], M6[2]]])
    assert np.allclose(mom.numpy(), M * dG, rtol=1e-10, atol=1e-10 * np.abs(M * dG).max())


def test_energy_and_wavespeed():
    w = make_workload("c1", n=3, N=3)
    S = from_workload(w)
    U = S.project(w.ic)
    # plane P wave: rho v^2/2 + (lambda+2mu) eps^2/2 = (lambda+2mu) A^2 sin^2, mean A^2/2
    A, lam2mu = 1e-6, 3 * 3.24e10
    want = lam2mu * A * A * 1000.0 ** 3 / 2
    assert abs(energy(S, U) - want) < 2e-3 * want
    assert torch.all(wavespeed_change(S, U) == 0)
    U[:, 0, 9] = 0.1 * math.sqrt(6.0)          # cell mean alpha = 0.6 -> clamped 0.5
    dc = wavespeed_change(S, U)
    assert torch.allclose(dc, torch.full_like(dc, math.sqrt((3.24e10 - 0.5 * 0.75 * 37e9) / 3.24e10) - 1))
