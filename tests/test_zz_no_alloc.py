"""dgd_energy_noalloc (the entry point for callers that cannot allocate device
memory) against dgd_energy, through the C-ABI.

Both run the same kernels on the same state; the partial sums of the first
live in the library's static device buffer, those of the second in memory
allocated per call, so the results agree to the last bit.  Two calls in a row
on different meshes, the second smaller (the buffer keeps the first call's
partial sums beyond the second mesh's elements; they must not leak into the
second result), in FP64 and FP32; a mesh above the buffer's 2^20 elements is
refused.
"""
import numpy as np
import pytest
import torch

from workloads import make_workload

pytestmark = pytest.mark.gpu


def _api():
    from paper_2502_09714_amd import api
    return api


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_noalloc_matches_energy(prec):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n, steps in ((5, 3), (3, 2)):                 # 750 tets, then 162
        w = make_workload("c2", n=n, N=3)
        sim = _api().from_workload(w, prec)
        sim.step(steps)
        want = sim.energy()
        sim.energy_noalloc(out)
        torch.cuda.synchronize()
        got = float(out.item())
        print(prec, w.ne, got, want, flush=True)
        assert np.isfinite(want) and want > 0
        assert got == want, (got, want)
        sim.close()


def test_energy_noalloc_refuses_large_meshes():
    from paper_2502_09714_amd._lib import DGDError
    w = make_workload("c2", n=56, N=1)              # 1,053,696 tets > 2^20
    assert w.ne > (1 << 20)
    sim = _api().Simulation(1, "fp32")
    m = w.mesh
    sim.set_mesh(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"])
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(DGDError, match="at most 1048576"):
        sim.energy_noalloc(out)
    sim.close()
