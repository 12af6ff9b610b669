"""Misfit gradients on the differentiation-form workload: 24^3 cubes x 6 =
82,944 tetrahedra, N = 3, 2 Hz Ricker double-couple point source 3 km below the
free surface, 16 receivers near the top face, 400 steps, checkpoints every 20
steps.  Misfit J = 1/2 sum |v - v_obs|^2 over all receivers and steps, v_obs
from the same run with mu0 perturbed by 5 % and C_d by 20 % per element (seeded).

The FP32 and FP64 adjoint gradients with respect to per-element mu0 and C_d
are checked against central finite differences of the FP64 forward run
(relative step 1e-4) on elements chosen without looking at the gradient: 20
drawn at random per parameter, plus the element holding the source, one
under a receiver (a free-surface face), one on an absorbing face and one on
an absorbing edge.  Bar per element: |g - fd| <= 1e-4 |fd| + a max|fd|, with
a = 1e-6 for the FP64 adjoint and 1e-5 for the FP32 one (the absolute part
covers elements the misfit hardly sees, whose difference quotient carries the
forward run's rounding, and the FP32 adjoint's own rounding).
"""
import numpy as np
import pytest

from workloads import make_workload
from workloads.configs import perturbed_material

pytestmark = pytest.mark.gpu

STEPS, EVERY = 400, 20


def _run(sim, U0, mat, n):
    sim.set_material(**mat)
    sim.set_state(U0)
    sim.set_time(0.0)
    sim.clear_seismograms()
    sim.step(n)
    return sim.get_seismograms()


@pytest.fixture(scope="module")
def c4():
    from paper_2502_09714_amd import api
    w = make_workload("c4")
    assert w.ne == 82944 and w.N == 3 and w.nsteps == STEPS and len(w.receivers) == 16
    base = {k: np.array(v, dtype=np.float64) for k, v in w.material.items()}
    s64 = api.from_workload(w, "fp64")
    U0 = s64.get_state()
    obs = _run(s64, U0, perturbed_material(base, seed=2), STEPS)
    assert np.abs(obs).max() > 0
    grads = {}
    for prec in ("fp64", "fp32"):
        sim = s64 if prec == "fp64" else api.from_workload(w, "fp32")
        sim.set_material(**base)
        sim.set_state(U0)
        sim.set_time(0.0)
        sim.clear_seismograms()
        sim.forward_checkpointed(STEPS, EVERY)
        seis = sim.get_seismograms()
        grads[prec] = sim.backward(seis - obs)
        if sim is not s64:
            sim.close()
    yield w, s64, U0, obs, base, grads
    s64.close()


def _misfit(s64, U0, obs, mat):
    seis = _run(s64, U0, mat, STEPS)
    return 0.5 * float(((seis - obs) ** 2).sum())


def _locate(w, x):
    """Element of the structured mesh containing point x (its cube, then the
    tetrahedron whose barycentric coordinates are all non-negative)."""
    m = w.mesh
    n, h = m["n"], m["edge"]
    o = m["xyz"].min(axis=0)
    ijk = np.minimum(((np.asarray(x) - o) // h).astype(int), n - 1)
    cube = ijk[0] + n * (ijk[1] + n * ijk[2])
    for e in range(6 * cube, 6 * cube + 6):
        X = m["xyz"][m["tets"][e]]
        lam = np.linalg.solve((X[1:] - X[0]).T, np.asarray(x) - X[0])
        if lam.min() >= -1e-12 and lam.sum() <= 1 + 1e-12:
            return e
    raise AssertionError("point outside its cube")


def _chosen_elements(w, seed):
    tag = w.mesh["face_tag"]
    rng = np.random.default_rng(seed)
    picks = [int(e) for e in rng.choice(w.ne, 20, replace=False)]
    picks.append(_locate(w, w.sources["xyz"][0]))                   # source host
    picks.append(_locate(w, w.receivers[5]))                        # under a receiver
    picks.append(int(np.nonzero((tag == 2).sum(1) == 1)[0][w.ne // 7 % 100]))   # absorbing face
    picks.append(int(np.nonzero((tag == 2).sum(1) >= 2)[0][0]))     # absorbing edge
    return list(dict.fromkeys(picks))


@pytest.mark.parametrize("which", ["mu0", "Cd"])
def test_c4_gradient_central_differences(c4, which):
    w, s64, U0, obs, base, grads = c4
    k = 0 if which == "mu0" else 1
    g64, g32 = grads["fp64"][k], grads["fp32"][k]
    assert np.isfinite(g64).all() and np.isfinite(g32).all()
    idx = _chosen_elements(w, 17 + k)
    fd = []
    for e in idx:
        h = 1e-4 * base[which][e]
        mp = {q: v.copy() for q, v in base.items()}
        mp[which][e] += h
        jp = _misfit(s64, U0, obs, mp)
        mp[which][e] -= 2 * h
        jm = _misfit(s64, U0, obs, mp)
        fd.append((jp - jm) / (2 * h))
    fd = np.asarray(fd)
    assert np.abs(fd).max() > 0
    for g, name, floor in ((g64[idx], "fp64", 1e-6), (g32[idx], "fp32", 1e-5)):
        bad = np.abs(g - fd) > 1e-4 * np.abs(fd) + floor * np.abs(fd).max()
        assert not bad.any(), (which, name, np.asarray(idx)[bad], g[bad], fd[bad])


def test_c4_fp32_adjoint_matches_fp64(c4):
    _, _, _, _, _, grads = c4
    for k in range(2):
        a, b = grads["fp32"][k], grads["fp64"][k]
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-4
