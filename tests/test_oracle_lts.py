"""Pins of the clustered local-time-stepping oracle (oracle/lts.py).

* One cluster: the scheme is the global step (the oracle's own step).
* Cluster construction: rate-2 clusters from the per-element admissible step,
  face neighbours at most one cluster apart, every element's step within its
  own admissible step.
* Conservation: on a periodic mesh with three clusters (the soft basin over
  rock: wave speeds 1200 and 6000 m/s) the wave quantities summed over the
  mesh do not change over a macro step (each face flux is computed once and
  used by both sides).
* A uniform state stays uniform across cluster boundaries.
* The elastic plane P wave (closed form) on a mesh whose half x < l/2 steps
  at twice the step of the other half: its error after a fixed time is that
  of the global step with the small step to within 10 %, and it falls at the
  design order N + 1 when the mesh is refined.
"""
import math

import numpy as np
import torch

from oracle.lts import LtsSolver, admissible_steps, make_clusters
from oracle.refmat import RefElement
from oracle.step import from_workload as oracle_from
from workloads import make_workload, plane_wave_ic


def test_single_cluster_is_the_global_step():
    w = make_workload("c2", n=3, N=2)
    S = oracle_from(w)
    U = S.project(w.ic)
    lts = LtsSolver(S, np.zeros(S.E, dtype=np.int64), w.dt)
    got = lts.macro_step(U)
    want = S.step(U)
    assert float((got - want).abs().max()) <= 1e-14 * float(want.abs().max())


def test_clusters_respect_the_rules():
    w = make_workload("c2", n=4, N=2, periodic=True)
    S = oracle_from(w)
    dte = admissible_steps(S)
    cl, dt0 = make_clusters(dte, S.mesh.nbr, 3)
    # the soft basin could take 4 dt_0 (wave speeds 1200 vs 6000 m/s), but its
    # one-element layer touches rock everywhere: one cluster above the rock
    slow = dte > 4 * dt0
    assert slow.any() and np.all(cl[slow] == 1) and np.all(cl[~slow] == 0)
    assert np.all(dt0 * 2.0 ** cl <= dte * (1 + 1e-12))
    # on their own the slow elements would go two clusters up
    lone, _ = make_clusters(dte, -np.ones_like(S.mesh.nbr), 3)
    assert np.all(lone[slow] == 2)
    nb = S.mesh.nbr
    has = nb >= 0
    assert np.abs(cl[np.maximum(nb, 0)] - cl[:, None])[has].max() <= 1
    # the global rule of the workloads is the fastest element's
    assert abs(dt0 - w.dt) < 1e-12 * w.dt


def _sums(S, U):
    vol = S.mesh.detJ
    return (vol[:, None] * U[:, 0, :9]).sum(0), (vol[:, None] * U[:, 0, :9].abs()).sum(0)


def test_conservation_across_clusters():
    w = make_workload("c2", n=4, N=2, periodic=True)
    w.material["Cd"] = np.zeros(w.ne)
    S = oracle_from(w)
    cl, dt0 = make_clusters(admissible_steps(S), S.mesh.nbr, 3)
    lts = LtsSolver(S, cl, dt0)
    U = S.project(w.ic)
    U1 = lts.macro_step(U)
    t0, s0 = _sums(S, U)
    t1, s1 = _sums(S, U1)
    assert bool(((t1 - t0).abs() <= 1e-12 * torch.maximum(s0, s1)).all())
    assert float((U1[:, :, :9] - U[:, :, :9]).abs().max()) > 0


def test_uniform_state_across_clusters():
    w = make_workload("c1", n=3, N=2)
    S = oracle_from(w)
    cent = w.mesh["xyz"][w.mesh["tets"]].mean(axis=1)
    cl = (cent[:, 0] < 500.0).astype(np.int64)
    lts = LtsSolver(S, cl, w.dt / 2)
    phi0 = float(S.ref.V[0, 0])
    U = torch.zeros((S.E, S.ref.L, 10), dtype=torch.float64)
    U[:, 0, :9] = torch.tensor([1e-5, -2e-5, 3e-6, 4e-6, 1e-6, -2e-6, 0.01, -0.02, 0.03],
                               dtype=torch.float64) / phi0
    U1 = lts.macro_step(U)
    assert float((U1 - U).abs().max()) <= 1e-13 * float(U.abs().max())


def _plane_wave_error(n, N, clustered, T):
    w = make_workload("c1", n=n, N=N)
    S = oracle_from(w)
    cent = w.mesh["xyz"][w.mesh["tets"]].mean(axis=1)
    dt_small = w.dt / 2
    nmacro = int(round(T / (2 * dt_small)))
    U = S.project(w.ic)
    if clustered:
        cl = (cent[:, 0] < 0.5 * w.mesh["length"]).astype(np.int64)
        out = LtsSolver(S, cl, dt_small).run(U, nmacro)
    else:
        S.dt = dt_small
        out = S.run(U, 2 * nmacro)
    t = nmacro * 2 * dt_small
    cp = w.extra["cp"]
    ic = plane_wave_ic(w.mesh["length"], w.extra["amplitude"], cp)
    exact = S.project(lambda x, elem=None: ic(x - np.array([cp * t, 0.0, 0.0])))
    return float(torch.linalg.norm(out - exact) / torch.linalg.norm(exact))


def test_plane_wave_with_a_clustered_half():
    N, T = 1, 0.02
    e3 = _plane_wave_error(3, N, True, T)
    g3 = _plane_wave_error(3, N, False, T)
    e6 = _plane_wave_error(6, N, True, T)
    rate = math.log2(e3 / e6)
    print(f"LTS {e3:.3e} (global step {g3:.3e}), refined {e6:.3e}, order {rate:.2f}")
    assert abs(e3 - g3) <= 0.1 * g3
    assert rate >= N + 0.5


def test_clusters_of_a_mesh_graded_around_a_fault():
    """The c5 recipe on a mesh whose band of layers around the fault is 8 times
    thinner: the band takes the smallest step, the coarse rock above and below
    at least twice it, and the global rule of the workload is the band's."""
    w = make_workload("c5f", n=12, N=2)
    S = oracle_from(w)
    assert bool((S.mesh.detJ > 0).all())
    z = w.mesh["z_nodes"]
    dz = np.diff(z)
    thin = dz < 0.5 * dz.max()
    assert thin.sum() == 2 and abs(dz[thin][0] * 8 - dz.max()) < 1e-9 * dz.max()
    dte = admissible_steps(S)
    cl, dt0 = make_clusters(dte, S.mesh.nbr, 8)
    assert abs(dt0 - w.dt) < 1e-12 * w.dt
    cent = w.mesh["xyz"][w.mesh["tets"]].mean(axis=1)[:, 2]
    band = (cent > z[:-1][thin].min()) & (cent < z[1:][thin].max())
    assert np.all(cl[band] == 0)
    # coarse elements with no band neighbour step at least twice as long
    nb = S.mesh.nbr
    touches = np.array([band[nb[e][nb[e] >= 0]].any() for e in range(S.E)])
    assert np.all(cl[~band & ~touches] >= 1)
    assert np.all(dt0 * 2.0 ** cl <= dte * (1 + 1e-12))
