"""GPU parity of clustered local time stepping (dgd_set_clusters,
dgd_make_clusters, dgd_step_lts) against the oracle's (oracle/lts.py).

* One cluster is the global step, to the last bit.
* The library's proposed clusters equal the oracle's, computed independently
  from the per-element admissible steps (soft basin over rock).
* Macro steps with several clusters match the oracle per quantity group
  (relative L2, pointwise maximum, per element): the periodic basin with its
  clusters from the wave speeds, a bounded mesh with damage growth and a
  clustered half, and a mesh graded in depth around a fault (clusters from
  the element sizes); FP64 1e-10, FP32 1e-5, BF16 3e-3.
* The wave quantities are conserved across cluster boundaries on the device.
* A point source (the c4 double couple, Ricker moment rate) in a clustered
  mesh, with receivers: state and seismograms against the oracle.
* Refusals: neighbours two clusters apart, the Picard predictor.
"""
import numpy as np
import pytest
import torch

from oracle.lts import LtsSolver, admissible_steps, make_clusters
from oracle.refmat import RefElement
from oracle.step import from_workload as oracle_from
from workloads import make_workload

from _metrics import assert_within, errors

pytestmark = pytest.mark.gpu


def _api():
    from paper_2502_09714_amd import api
    return api


def _to_lib(U):
    return U.permute(0, 2, 1).contiguous().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_cluster_is_the_global_step(prec):
    w = make_workload("c2", n=3, N=3)
    a = _api().from_workload(w, prec)
    b = _api().from_workload(w, prec)
    b.set_clusters(np.zeros(w.ne, dtype=np.int32), w.dt)
    a.step(3)
    b.step_lts(3)
    assert np.array_equal(a.get_state(), b.get_state())
    assert abs(a.get_time() - b.get_time()) < 1e-15
    a.close()
    b.close()


def test_clusters_match_the_oracle():
    w = make_workload("c2", n=4, N=2, periodic=True)
    S = oracle_from(w)
    want, dt0 = make_clusters(admissible_steps(S), S.mesh.nbr, 3)
    sim = _api().from_workload(w, "fp64")
    got, gdt0 = sim.make_clusters(0.5, 3)
    assert np.array_equal(got, want) and abs(gdt0 - dt0) < 1e-14 * dt0
    assert got.max() == 1
    sim.close()


def _half(w):
    cent = w.mesh["xyz"][w.mesh["tets"]].mean(axis=1)
    return (cent[:, 0] < 0.5 * w.mesh["length"]).astype(np.int32)


CASES = [
    # periodic basin, clusters from the wave speeds
    ("basin", "c2", dict(n=4, N=2, periodic=True), 2),
    # bounded basin with damage growth, x < l/2 at twice the step
    ("half", "c2", dict(n=3, N=3), 2),
    # the mesh graded in depth around a fault (a band of layers 8 times
    # thinner), clusters from the element sizes and wave speeds, a plane P
    # wave through it
    ("band", "c5f", dict(n=6, N=2), 1),
]


def _band_workload(w):
    from workloads import plane_wave_ic
    w.sources = None
    w.receivers = None
    w.ic = plane_wave_ic(w.mesh["length"], 1e-5, 6000.0)
    return w


_ORACLE = {}


def _oracle_case(kind, name, kw, nmacro):
    """Workload, clusters, initial and final oracle states of a case (the
    oracle's run is shared by the precisions)."""
    key = (kind, name, tuple(sorted(kw.items())), nmacro)
    if key not in _ORACLE:
        w = make_workload(name, **kw)
        if kind == "band":
            w = _band_workload(w)
        S = oracle_from(w)
        if kind in ("basin", "band"):
            cl, dt0 = make_clusters(admissible_steps(S), S.mesh.nbr, 8 if kind == "band" else 3)
        else:
            cl, dt0 = _half(w), w.dt / 2
        U0 = S.project(w.ic)
        _ORACLE[key] = (w, cl, dt0, U0, LtsSolver(S, cl, dt0).run(U0, nmacro))
    return _ORACLE[key]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("kind,name,kw,nmacro", CASES)
def test_lts_parity(kind, name, kw, nmacro, prec, tol):
    w, cl, dt0, U0, want = _oracle_case(kind, name, kw, nmacro)
    if kind == "band":
        assert cl.max() >= 2 and (cl == 0).any()
    sim = _api().from_workload(w, prec, state=False)
    sim.set_state(_to_lib(U0))
    sim.set_clusters(cl, dt0)
    sim.step_lts(nmacro)
    e = errors(sim.get_state(), _to_lib(want), RefElement(w.N).V.numpy())
    print(kind, kw, prec, e, flush=True)
    assert_within(e, tol, f"LTS {kind} {prec}")
    assert abs(sim.get_time() - nmacro * dt0 * 2 ** int(cl.max())) < 1e-12
    sim.close()


def test_lts_conserves_on_the_device():
    w = make_workload("c2", n=4, N=2, periodic=True)
    w.material["Cd"] = np.zeros(w.ne)
    sim = _api().from_workload(w, "fp64")
    cl, dt0 = sim.make_clusters(0.5, 3)
    sim.set_clusters(cl, dt0)
    U0 = sim.get_state()
    sim.step_lts(2)
    U1 = sim.get_state()
    s0, s1 = U0[:, :9, 0].sum(0), U1[:, :9, 0].sum(0)     # uniform |J|
    scale = np.maximum(np.abs(U0[:, :9, 0]).sum(0), np.abs(U1[:, :9, 0]).sum(0))
    assert np.all(np.abs(s1 - s0) <= 1e-12 * scale)
    assert np.abs(U1[:, 6:9] - U0[:, 6:9]).max() > 0
    sim.close()


def test_lts_point_source_and_receivers():
    from oracle.sources import PointSources, Receivers
    w = make_workload("c4", n=4, N=2)
    S = oracle_from(w)
    xs = w.sources["xyz"][0]
    recx = xs[None, :] + np.array([[310.0, -170.0, 90.0], [40.0, 35.0, -25.0]])
    cl = _half(w)
    cl[:] = 0
    cent = w.mesh["xyz"][w.mesh["tets"]].mean(axis=1)
    cl[np.linalg.norm(cent - xs, axis=1) < 4000.0] = 1     # the source region at twice the step
    dt0 = w.dt / 2
    t0 = 0.45
    src = PointSources(S, **w.sources)
    rec = Receivers(S, recx)
    lts = LtsSolver(S, cl, dt0, sources=src)
    U = S.project(w.ic)
    want_seis = []
    for k in range(3):
        U = lts.macro_step(U, t0 + k * lts.macro_dt)
        want_seis.append(rec.sample(U).numpy())
    sim = _api().from_workload(w, "fp64", state=False)
    sim.set_receivers(recx)
    sim.set_state(_to_lib(S.project(w.ic)))
    sim.set_time(t0)
    sim.set_clusters(cl, dt0)
    sim.step_lts(3)
    e = errors(sim.get_state(), _to_lib(U), RefElement(w.N).V.numpy())
    assert_within(e, 1e-10, "LTS with a point source")
    got = sim.get_seismograms()
    want = np.stack(want_seis)
    assert np.abs(want).max() > 0
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10
    sim.close()


def test_lts_refusals():
    from paper_2502_09714_amd._lib import DGDError
    w = make_workload("c4", n=3, N=2)
    sim = _api().from_workload(w, "fp64")
    cl = np.zeros(w.ne, dtype=np.int32)
    cl[0] = 2
    with pytest.raises(DGDError, match="EINVAL"):
        sim.set_clusters(cl, w.dt)
    sim.set_clusters(np.zeros(w.ne, dtype=np.int32), w.dt)
    sim.set_predictor("picard")
    with pytest.raises(DGDError, match="EINVAL"):
        sim.step_lts(1)
    sim.set_predictor("ck")
    sim.step_lts(1)
    sim.close()
