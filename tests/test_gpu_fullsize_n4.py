"""Parity of one step of the degree-4 workloads at their full sizes:
c3 (64^3 cubes x 6 = 1,572,864 tetrahedra, layered basin with lognormal
moduli, 32 strain pulses) in FP64 and FP32, and c5 (96^3 cubes x 6 = 5,308,416
tetrahedra, the 3 km gradient basin, 24 km box) in FP32, the largest
configuration.  Sampled elements (random, plus a free-surface element and an
absorbing edge/corner element) against the oracle's step of the patch
{element, face neighbours}; bars as for the other parity tests, relative L2
per element 1e-10 (FP64) and 1e-5 (FP32).  The point sources of c5 are left
out (their parity is covered on the small cut); the step is the same kernels
at 8 times the element count of the benchmark workload.  The initial state is
projected on the device once per workload (chunk by chunk, with progress
lines) and handed to the other precision as modal coefficients.
"""
import numpy as np
import pytest

from _metrics import ELEM_FACTOR, element_errors, group_scales
from _patch import face_partners, oracle_patch_step
from workloads import make_workload

pytestmark = pytest.mark.gpu

SIZES = {"c3": (1572864, 4), "c5": (5308416, 4)}


def _setup(name):
    w = make_workload(name)
    assert (w.ne, w.N) == SIZES[name]
    w.sources = None
    w.receivers = None
    nbr = face_partners(w.mesh)
    rng = np.random.default_rng(321)
    sample = [int(e) for e in rng.choice(w.ne, 8, replace=False)]
    tag = w.mesh["face_tag"]
    sample.append(int(np.nonzero((tag == 1).any(1))[0][-1]))        # free surface
    sample.append(int(np.nonzero((tag == 2).sum(1) >= 2)[0][-1]))   # absorbing edge/corner
    want = {e: oracle_patch_step(w, e, nbr) for e in sample}
    return {"w": w, "sample": sample, "want": want, "U0": None}


def _sim(case, prec):
    from paper_2502_09714_amd import api
    w = case["w"]
    sim = api.from_workload(w, prec, state=False)
    if case["U0"] is not None:
        sim.set_state(case["U0"])
        return sim
    chunk = max(1, (1 << 22) // sim.Q)
    starts = list(range(0, sim.ne, chunk))
    for i, e0 in enumerate(starts):
        cnt = min(chunk, sim.ne - e0)
        x = sim.get_quadrature_points(e0, cnt)
        elem = np.repeat(np.arange(e0, e0 + cnt), sim.Q)
        sim.set_state_from_points(w.ic(x.reshape(-1, 3), elem), e0)
        if i % 8 == 7:
            print(f"  projected {e0 + cnt} of {sim.ne} elements", flush=True)
    case["U0"] = sim.get_state()
    return sim


@pytest.fixture(scope="module")
def cases():
    return {}


@pytest.mark.parametrize("name,prec,tol", [("c3", "fp64", 1e-10), ("c3", "fp32", 1e-5),
                                           ("c3", "bf16", 3e-3), ("c5", "fp32", 1e-5),
                                           ("c5", "bf16", 3e-3)])
def test_fullsize_degree4_sampled_parity(cases, name, prec, tol):
    if name not in cases:
        cases.clear()                      # one workload's host arrays at a time
        cases[name] = _setup(name)
    case = cases[name]
    w, sample, want = case["w"], case["sample"], case["want"]
    print(f"{name} {prec}: {w.ne} tets, N={w.N}, sampled {sample}", flush=True)
    sim = _sim(case, prec)
    print(f"{name} {prec}: state set, stepping", flush=True)
    sim.step(1)
    got = sim.get_state()
    sim.close()
    print(f"{name} {prec}: stepped", flush=True)
    assert np.isfinite(got).all()
    sc = group_scales(got)
    for e in sample:
        r = element_errors(got[e].T, want[e], sc)          # (L, 10) each
        print(f"  element {e}: {r}", flush=True)
        assert max(r.values()) < ELEM_FACTOR * tol, (name, prec, e, r)
