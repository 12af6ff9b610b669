"""Misfit gradients on the differentiation-form workload: 24^3 cubes x 6 =
82,944 tetrahedra, N = 3, 2 Hz Ricker double-couple point source 3 km below the
free surface, 16 receivers near the top face, 400 steps, checkpoints every 20
steps.  Misfit J = 1/2 sum |v - v_obs|^2 over all receivers and steps, v_obs
from the same run with mu0 perturbed by 5 % and C_d by 20 % per element (seeded).

The FP32 and FP64 adjoint gradients with respect to per-element mu0 and C_d
are checked against central finite differences of the FP64 forward run
(relative step 1e-4) on 10 seeded elements drawn among those the misfit is
sensitive to (|dJ/dp| at least 1e-3 of its maximum): relative L2 1e-4.
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


@pytest.mark.parametrize("which", ["mu0", "Cd"])
def test_c4_gradient_central_differences(c4, which):
    w, s64, U0, obs, base, grads = c4
    k = 0 if which == "mu0" else 1
    g64, g32 = grads["fp64"][k], grads["fp32"][k]
    assert np.isfinite(g64).all() and np.isfinite(g32).all()
    cand = np.nonzero(np.abs(g64) >= 1e-3 * np.abs(g64).max())[0]
    idx = np.random.default_rng(17 + k).choice(cand, 10, replace=False)
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
    r64 = np.linalg.norm(g64[idx] - fd) / np.linalg.norm(fd)
    r32 = np.linalg.norm(g32[idx] - fd) / np.linalg.norm(fd)
    assert r64 < 1e-4, (r64, g64[idx], fd)
    assert r32 < 1e-4, (r32, g32[idx], fd)


def test_c4_fp32_adjoint_matches_fp64(c4):
    _, _, _, _, _, grads = c4
    for k in range(2):
        a, b = grads["fp32"][k], grads["fp64"][k]
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-4
