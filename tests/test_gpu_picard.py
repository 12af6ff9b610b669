"""GPU parity of the Picard-iteration predictor (dgd_set_predictor) against
the oracle's (oracle/picard.py), and its effect on accuracy in time.

Parity: small cuts of the tiny periodic plane-wave configuration (N = 2), of
the layered basin with boundaries and damage growth (N = 3) and of the
lognormal precision-form configuration (N = 4), the IVM law, and the number of
iterations; every quantity group by relative L2, pointwise maximum and per
element, bars 1e-10 (FP64), 1e-5 (FP32), 3e-3 (BF16).

"""

import numpy as np
import pytest
import torch

from oracle.picard import picard_from_workload, predict_picard
from oracle.refmat import RefElement
from workloads import make_workload

from _metrics import assert_within, errors

pytestmark = pytest.mark.gpu


def _api():
    from paper_2502_09714_amd import api
    return api


def _to_lib(U):
    return U.permute(0, 2, 1).contiguous().numpy()


CASES = [
    ("c1", dict(n=3, N=2), 2, None),
    ("c2", dict(n=3, N=3), 2, None),
    ("c3", dict(n=3, N=4), 1, None),
    ("c2", dict(n=3, N=2), 2, 1),          # one sweep
    ("c2", dict(n=3, N=2), 2, 6),          # more sweeps than the default N + 1
]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("name,kw,nsteps,iters", CASES)
def test_picard_parity(name, kw, nsteps, iters, prec, tol):
    w = make_workload(name, **kw)
    S = picard_from_workload(w, iterations=iters)
    U0 = S.project(w.ic)
    sim = _api().from_workload(w, prec, state=False)
    sim.set_predictor("picard", 0 if iters is None else iters)
    sim.set_state(_to_lib(U0))
    sim.step(1)
    if prec == "fp64":
        got_z = sim.get_time_point_states()                       # (E, Nt, 10, L)
        want_z = predict_picard(S, U0, S.iterations).permute(1, 0, 3, 2).numpy()
        assert np.linalg.norm(got_z - want_z) / np.linalg.norm(want_z) < 1e-12
    U = S.run(U0, nsteps)
    sim.step(nsteps - 1)
    e = errors(sim.get_state(), _to_lib(U), RefElement(w.N).V.numpy())
    print(name, kw, iters, prec, e, flush=True)
    assert_within(e, tol, f"Picard {name} {kw} {prec}")
    sim.close()


def test_picard_ivm_law():
    w = make_workload("c2", n=3, N=3, rheology="ivm")
    S = picard_from_workload(w)
    U0 = S.project(w.ic)
    sim = _api().from_workload(w, "fp64", state=False)
    sim.set_predictor("picard")
    sim.set_state(_to_lib(U0))
    sim.step(2)
    e = errors(sim.get_state(), _to_lib(S.run(U0, 2)), RefElement(w.N).V.numpy())
    assert_within(e, 1e-10, "Picard IVM")
    sim.close()


def test_picard_refuses_the_adjoint():
    from paper_2502_09714_amd._lib import DGDError
    w = make_workload("c2", n=3, N=2)
    sim = _api().from_workload(w, "fp64")
    sim.set_predictor("picard")
    with pytest.raises(DGDError, match="EINVAL"):
        sim.forward_checkpointed(2, 1)
    sim.set_predictor("ck")
    sim.forward_checkpointed(2, 1)
    sim.close()
