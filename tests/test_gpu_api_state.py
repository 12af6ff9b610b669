"""Argument and state checks of the C-ABI (through the binding, on the GPU).

* The clamp alpha_max must leave the boundary moduli positive for every
  admissible state: under the CDM law mu_eff = mu0 + a xi0 gamma_r -
  a gamma_r xi/2 and lambda_eff + 2 mu_eff (Eq. effective-cdb, reading R4)
  over a in [0, alpha_max], xi in [-sqrt 3, sqrt 3]; under the IVM law
  alpha_max < 1 (Eq. ivm-model is singular at alpha = 1).
* A checkpointed run is dropped by every call that changes the problem; the
  backward sweep then reports DGD_ESTATE instead of replaying the run with
  the new definition.
"""
import math

import numpy as np
import pytest
import torch

from workloads import make_workload

pytestmark = pytest.mark.gpu


def _api():
    from paper_2502_09714_amd import api
    return api


def _err():
    from paper_2502_09714_amd._lib import DGDError
    return DGDError


def _largest_admissible_amax(mat):
    """Largest alpha_max keeping both CDM boundary moduli positive (closed
    form of the corner conditions, per element, minimised)."""
    mu, lam, gr, xi0 = mat["mu0"], mat["lambda0"], mat["gamma_r"], mat["xi0"]
    r3 = math.sqrt(3.0)
    bounds = []
    for xi in (-r3, r3):
        s_mu = -(xi0 * gr - 0.5 * gr * xi)          # mu_eff = mu - a * s_mu
        s_pm = -(2 * xi0 * gr - 4.0 / 3.0 * gr * xi)
        for base, slope in ((mu, s_mu), (lam + 2 * mu, s_pm)):
            with np.errstate(divide="ignore"):
                bounds.append(np.where(slope > 0, base / slope, np.inf))
    return float(np.min(bounds))


def test_alpha_max_validation_cdm():
    w = make_workload("c1", n=3, N=1)
    amax_ok = _largest_admissible_amax(w.material)
    assert 0.5 < amax_ok < 1.0            # Table 1 moduli: about 0.54
    sim = _api().from_workload(w, "fp64")
    sim.set_params(w.dt, 0.999 * amax_ok)
    with pytest.raises(_err(), match="EINVAL"):
        sim.set_params(w.dt, 1.001 * amax_ok)
    sim.set_params(w.dt, 0.5)
    # a material that the current clamp makes non-positive is refused
    bad = dict(sim.material)
    bad["gamma_r"] = bad["gamma_r"].copy()
    bad["gamma_r"][7] *= 3.0
    with pytest.raises(_err(), match="EINVAL"):
        sim.set_material(**bad)
    sim.step(1)                           # the old material is still in place
    sim.synchronize()
    sim.close()


def test_alpha_max_validation_ivm():
    w = make_workload("c1", n=3, N=1, rheology="ivm")
    sim = _api().from_workload(w, "fp64")
    with pytest.raises(_err(), match="EINVAL"):
        sim.set_params(w.dt, 1.0)
    sim.set_params(w.dt, 0.99)
    sim.close()


def test_tape_dropped_by_problem_changes():
    w = make_workload("c2", n=3, N=1)
    sim = _api().from_workload(w, "fp64")
    m = w.mesh
    cent = m["xyz"][m["tets"][[5, 40]]].mean(axis=1)
    sim.set_receivers(cent)
    U0 = sim.get_state()
    mat = dict(sim.material)

    def record():
        sim.set_state(U0)
        sim.clear_seismograms()
        sim.forward_checkpointed(3, 2)
        return sim.get_seismograms()

    changes = [
        lambda: sim.set_material(**mat),
        lambda: sim.set_params(w.dt, w.alpha_max),
        lambda: sim.set_receivers(cent),
        lambda: sim.set_point_sources(cent[:1], np.array([[1e12, 0, 0, 0, 0, 0]]), [0.0], [0.1], 1),
    ]
    ids = []
    for change in changes:
        seis = record()
        tid = sim.tape_id()
        assert tid > 0 and tid not in ids
        ids.append(tid)
        sim.backward(seis)                # the tape is there
        change()
        assert sim.tape_id() == 0
        with pytest.raises(_err(), match="ESTATE"):
            sim.backward(seis)
    sim.set_point_sources(np.zeros((0, 3)), np.zeros((0, 6)), [], [], 0)
    # a new mesh with more elements: no replay from the old, smaller checkpoints
    seis = record()
    w2 = make_workload("c2", n=4, N=1)
    m2 = w2.mesh
    sim.set_mesh(m2["xyz"], m2["tets"], m2["face_tag"], m2["periodic_map"])
    assert sim.tape_id() == 0
    with pytest.raises(_err(), match="ESTATE"):
        sim.backward(seis)
    sim.close()


def test_autograd_refuses_a_stale_tape():
    from paper_2502_09714_amd.adjoint import seismograms
    w = make_workload("c2", n=3, N=1)
    m = w.mesh
    cent = m["xyz"][m["tets"][[5, 40]]].mean(axis=1)
    sim = _api().from_workload(w, "fp64")
    sim.set_receivers(cent)
    U0 = sim.get_state()
    mu0 = torch.tensor(w.material["mu0"], requires_grad=True)
    cd = torch.tensor(w.material["Cd"], requires_grad=True)
    s1 = seismograms(sim, mu0, cd, U0, nsteps=2, every=1)
    s2 = seismograms(sim, mu0 * 1.01, cd, U0, nsteps=2, every=1)
    with pytest.raises(RuntimeError, match="checkpointed run"):
        s1.sum().backward()
    s2.sum().backward()                   # the graph of the kept run works
    assert torch.isfinite(mu0.grad).all()
    sim.close()
