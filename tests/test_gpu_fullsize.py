"""Parity at the full benchmark size, in the launch configuration bench.py
times: the 663,552-tetrahedron degree-3 layered-basin workload (48^3 cubes x 6,
free top, absorbing sides, 32 strain pulses, damage alpha0 ~ U(0, 0.05)).

One GPU step of the whole mesh; sampled elements (random, plus free-surface,
absorbing-corner and basin-interface elements) against the oracle's step of
the patch {element, face neighbours}, which the CPU test of the patch helper
ties to the whole-mesh oracle.  Bars: relative L2 per element 1e-10 (FP64),
1e-5 (FP32).  Whole-mesh properties at full size: a finite state, FP32 within
1e-5 of FP64, and a rest state (zero strain and velocity, damage varying
between elements) keeps its wave quantities exactly zero while the
Lax-Friedrichs term only exchanges damage between elements (its total, on
this uniform mesh with no damage flux through the boundary, is conserved).
"""
import numpy as np
import pytest

from _patch import face_partners, oracle_patch_step
from _metrics import ELEM_FACTOR, element_errors, group_scales
from workloads import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    w = make_workload("c2")
    assert w.ne == 663552 and w.N == 3
    nbr = face_partners(w.mesh)
    rng = np.random.default_rng(123)
    sample = list(rng.choice(w.ne, 12, replace=False))
    tag = w.mesh["face_tag"]
    sample.append(int(np.nonzero((tag == 1).any(1))[0][0]))         # free surface
    sample.append(int(np.nonzero((tag == 2).sum(1) >= 2)[0][0]))    # absorbing edge/corner
    mu = w.material["mu0"]
    jump = np.nonzero([(nbr[e] >= 0).any() and (mu[nbr[e][nbr[e] >= 0]] != mu[e]).any()
                       for e in range(0, w.ne, 97)])[0]
    sample.append(int(jump[0] * 97))                                 # basin interface
    want = {e: oracle_patch_step(w, e, nbr) for e in sample}
    return w, sample, want


def _gpu_step(w, prec):
    from paper_2502_09714_amd import api
    sim = api.from_workload(w, prec)
    sim.step(1)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16", 3e-3)])
def test_fullsize_sampled_parity(big, prec, tol):
    w, sample, want = big
    got = _gpu_step(w, prec)
    assert np.isfinite(got).all()
    sc = group_scales(got)
    for e in sample:
        r = element_errors(got[e].T, want[e], sc)
        print(f"  element {e}: {r}", flush=True)
        assert max(r.values()) < ELEM_FACTOR * tol, (prec, e, r)


def test_fullsize_precisions_and_rest_state(big):
    w, _, _ = big
    from paper_2502_09714_amd import api
    a = _gpu_step(w, "fp64")
    b = _gpu_step(w, "fp32")
    assert np.linalg.norm(b - a) / np.linalg.norm(a) < 1e-5
    # rest state with damage: no strain, no velocity -> nothing moves
    sim = api.from_workload(w, "fp32", state=False)
    z = np.zeros((w.ne, 10, sim.L))
    z[:, 9, 0] = np.random.default_rng(1).uniform(0.0, 0.3, w.ne)
    sim.set_state(z)
    sim.step(2)
    out = sim.get_state()
    sim.close()
    assert np.abs(out[:, :9]).max() == 0.0
    assert not np.array_equal(out[:, 9], z[:, 9])
    assert abs(out[:, 9, 0].sum() - z[:, 9, 0].sum()) <= 1e-6 * z[:, 9, 0].sum()
