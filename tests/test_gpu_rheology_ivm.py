"""GPU parity of the internal-variable rheology (Eq. ivm-model, Murnaghan
terms off, boundary moduli of Eq. effective-ivm) against the oracle with the
same law: small cuts of the c1 (periodic, N = 2), c2 (layered basin, free top,
absorbing sides, N = 3) and c3 (lognormal moduli, N = 4) recipes with the IVM
parameters of ``workloads.ivm_material`` (damage grows in strained rock and
heals in the basin, where the storage energy of the initial damage exceeds the
strain energy).  A fourth case keeps Table 2's damage time scale tau_b = 10 s
(the other cases shorten it so that damage moves within a few steps).  Every
quantity group is checked by relative L2, pointwise maximum and per element
(tests/_metrics.py).  Bars: 1e-10 (FP64), 1e-5 (FP32), 3e-3 (BF16 matrix-core
inputs, FP32 accumulation).
"""
import numpy as np
import pytest

from oracle.diagnostics import wavespeed_change as oracle_dcs
from oracle.step import from_workload as oracle_from
from oracle.refmat import RefElement
from workloads import make_workload
from workloads.configs import ivm_material

from _metrics import assert_within, errors

pytestmark = pytest.mark.gpu

CASES = {
    "c1": (dict(n=4, N=2), 4),
    "c2": (dict(n=3, N=3), 3),
    "c3": (dict(n=3, N=4), 2),
    "c2_table2": (dict(n=3, N=3), 3),
}
_cache = {}


def _oracle(name):
    if name not in _cache:
        kw, nsteps = CASES[name]
        w = make_workload(name.split("_")[0], rheology="ivm", **kw)
        if name.endswith("table2"):
            base = make_workload("c2", **kw).material
            w.material = ivm_material(base, tau_b=10.0)
        S = oracle_from(w)
        assert S.law.__name__.endswith("ivm")
        U0 = S.project(w.ic)
        U1 = S.run(U0, nsteps)
        _cache[name] = (w, S, U0, U1, nsteps)
    return _cache[name]


def _to_lib(U):
    return U.permute(0, 2, 1).contiguous().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,prec,tol", [
    ("c1", "fp64", 1e-10), ("c2", "fp64", 1e-10), ("c3", "fp64", 1e-10),
    ("c2_table2", "fp64", 1e-10),
    ("c1", "fp32", 1e-5), ("c2", "fp32", 1e-5), ("c3", "fp32", 1e-5),
    ("c2_table2", "fp32", 1e-5),
    ("c1", "bf16", 3e-3), ("c2", "bf16", 3e-3), ("c3", "bf16", 3e-3)])
def test_ivm_step_parity(name, prec, tol):
    from paper_2502_09714_amd import api
    w, S, U0, U1, nsteps = _oracle(name)
    want = _to_lib(U1)
    # the damage moved, both ways in the layered cases
    da = U1[:, 0, 9] - U0[:, 0, 9]
    # tau_b = 10 s: the damage still moves, at a rate 1e5 times smaller
    assert float(da.abs().max()) > (1e-11 if name.endswith("table2") else 1e-6)
    if name in ("c2", "c3"):
        assert float(da.max()) > 0 and float(da.min()) < 0
    sim = api.from_workload(w, prec, state=False)
    sim.set_state(_to_lib(U0))
    sim.step(nsteps)
    got = sim.get_state()
    assert np.isfinite(got).all()
    e = errors(got, want, RefElement(w.N).V.numpy())
    print(name, prec, e, flush=True)
    assert_within(e, tol, f"IVM {name} {prec}")
    # the damage change itself, not only the damage, to the bar
    dgot = got[:, 9] - _to_lib(U0)[:, 9]
    dwant = want[:, 9] - _to_lib(U0)[:, 9]
    assert _rel(dgot, dwant) < (tol if prec != "fp32" or not name.endswith("table2") else 1e-3)
    if prec == "fp64":
        # damage-only shear-wave-speed change sqrt(1 - abar) - 1
        d = sim.wavespeed_change()
        assert np.allclose(d, oracle_dcs(S, U1).numpy(), rtol=0, atol=1e-13)
    sim.close()


def test_ivm_rejects_cdm_only_calls():
    from paper_2502_09714_amd import api
    from paper_2502_09714_amd._lib import DGDError
    w, _, U0, _, _ = _oracle("c2")
    sim = api.from_workload(w, "fp32", state=False)
    sim.set_state(_to_lib(U0))
    for call in (sim.energy, lambda: sim.forward_checkpointed(2, 1)):
        with pytest.raises(DGDError):
            call()
    bad = dict(w.material)
    with pytest.raises(DGDError):
        sim.set_material_ivm(bad["rho"], bad["lambda0"], bad["mu0"], -bad["gamma_b"], bad["tau_b"])
    sim.close()
