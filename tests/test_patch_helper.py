"""The single-element oracle patch used by the full-size GPU parity test
reproduces the whole-mesh oracle step exactly (periodic and bounded meshes)."""
import numpy as np
import pytest

from _patch import face_partners, oracle_patch_step
from oracle.step import from_workload as oracle_from
from workloads import make_workload


@pytest.mark.parametrize("name", ["c2", "c1"])
def test_patch_step_equals_full_oracle(name):
    w = make_workload(name, n=3, N=2)
    S = oracle_from(w)
    U1 = S.step(S.project(w.ic)).detach().numpy()
    nbr = face_partners(w.mesh)
    assert np.array_equal(nbr, S.mesh.nbr)
    for e in (0, 17, 101, w.ne - 1):
        u = oracle_patch_step(w, e, nbr)
        assert np.abs(u - U1[e]).max() <= 1e-13 * np.abs(U1[e]).max()
