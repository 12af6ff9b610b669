"""FP32 and split-BF16 against the FP64 GPU path over 20 steps of the whole
degree-4 precision-form mesh (c3: 64^3 cubes x 6 = 1,572,864 tetrahedra,
layered basin with lognormal moduli, 32 strain pulses, no sources), from the
same FP64 state, in the launch configuration bench.py times.

Every quantity group (strain, velocity, alpha) is checked by relative L2 over
the mesh, by max |error| / max |value| over the volume quadrature points and
per element (tests/_metrics.py); bars 1e-5 (FP32) and 3e-3 (BF16 matrix-core
inputs, FP32 accumulation).  The FP64 path itself is tied to the oracle on
sampled elements of the same mesh (test_gpu_fullsize_n4.py).
"""
import numpy as np
import pytest

from _metrics import assert_within, errors
from oracle.refmat import RefElement
from workloads import make_workload

pytestmark = pytest.mark.gpu

STEPS = 20


def test_c3_fullsize_mixed_forms_against_fp64():
    from paper_2502_09714_amd import api
    w = make_workload("c3")
    assert (w.ne, w.N) == (1572864, 4)
    w.sources = None
    w.receivers = None
    ref = api.from_workload(w, "fp64")
    ref.set_check_interval(1 << 40)
    U0 = ref.get_state()
    print(f"c3: {w.ne} tets projected; FP64 {STEPS} steps", flush=True)
    ref.step(STEPS)
    want = ref.get_state()
    ref.close()
    assert np.isfinite(want).all()
    V = RefElement(w.N).V.numpy()
    for prec, tol in (("fp32", 1e-5), ("bf16", 3e-3)):
        sim = api.from_workload(w, prec, state=False)
        sim.set_check_interval(1 << 40)
        sim.set_state(U0)
        sim.step(STEPS)
        got = sim.get_state()
        sim.close()
        e = errors(got, want, V)
        print(f"c3 {prec} after {STEPS} steps: {e}", flush=True)
        assert_within(e, tol, f"c3 {prec}")
