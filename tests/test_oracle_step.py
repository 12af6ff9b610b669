"""Pins of the oracle's full ADER-DG step.

* a uniform state is steady (C_d = 0), or its damage grows exactly linearly
  at the closed-form rate r_alpha = C_d gamma_r I2 (xi - xi0) (C_d > 0);
* on a periodic mesh the element integrals of the nine wave quantities are
  conserved and the total damage changes exactly by the integrated source;
* energy does not increase while damage grows;
* in the elastic limit a plane P wave is transported at c_p: the error
  against the analytic solution is small and drops with the polynomial
  degree on a fixed mesh (p-convergence, Section 3.1);
* face points matched through the neighbour map coincide physically;
* brute force on one element: the matrix form of the predictor's first
  derivative, the volume integral and the face integral equals a direct
  high-order quadrature written with plain loops (exact in the elastic limit).
"""
import math

import numpy as np
import pytest
import torch
from scipy.special import roots_jacobi

from oracle import boundary, cdm
from oracle.refmat import FACE_VERTS, face_to_ref
from oracle.step import OracleSolver, from_workload
from workloads import make_workload, plane_wave_ic
from workloads.mesh import cube_mesh

DT = torch.float64


def _homog(ne, Cd=0.0):
    f = lambda v: np.full(ne, v)
    return dict(rho=f(2700.0), lambda0=f(2.0e10), mu0=f(1.5e10), gamma_r=f(1.7e10),
                xi0=f(-0.75), Cd=f(Cd))


def _solver(n=3, N=2, periodic=True, mat=None, dt=1e-3, **kw):
    m = cube_mesh(n, 900.0, periodic=periodic)
    ne = m["tets"].shape[0]
    return OracleSolver(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"],
                        mat if mat is not None else _homog(ne), N, dt, **kw)


def _uniform_state(S, seed=0):
    rng = np.random.default_rng(seed)
    val = np.concatenate([rng.standard_normal(6) * 1e-4, rng.standard_normal(3), [0.2]])
    return S.project(lambda x, e: np.tile(val, (x.shape[0], 1))), val


def test_uniform_state_is_steady():
    S = _solver()
    U, _ = _uniform_state(S)
    U1 = S.step(U)
    assert float(torch.linalg.norm(U1 - U) / torch.linalg.norm(U)) < 1e-14


def test_uniform_damage_growth_closed_form():
    S = _solver(mat=_homog(162, Cd=1e-2), dt=2e-3)
    U, val = _uniform_state(S, seed=1)
    e = val[:6]
    I1 = e[:3].sum()
    I2 = (e[:3] ** 2).sum() + 2 * (e[3:] ** 2).sum()
    xi = I1 / math.sqrt(I2)
    r = 1e-2 * 1.7e10 * I2 * (xi + 0.75) if xi > -0.75 else 0.0
    assert r > 0
    U1 = S.step(U)
    want = U.clone()
    want[:, 0, 9] += S.dt * r * math.sqrt(6.0) / 6.0     # int phi_0 = sqrt(6)/6
    assert torch.allclose(U1, want, rtol=0, atol=1e-14 * float(U.abs().max()))


def _random_smooth(S, seed):
    g = torch.Generator().manual_seed(seed)
    U = torch.randn(S.E, S.ref.L, 10, generator=g, dtype=DT)
    U[..., :6] *= 1e-5
    U[..., 6:9] *= 1e-2
    U[..., 9] = 0.05 * torch.rand(S.E, S.ref.L, generator=g, dtype=DT)
    U[:, 1:, :] *= 0.2
    return U


def test_conservation_periodic():
    rng = np.random.default_rng(3)
    mat = _homog(162, Cd=1e-2)
    mat["gamma_r"] = mat["gamma_r"] * (1 + 0.3 * rng.random(162))
    mat["mu0"] = mat["mu0"] * (1 + 0.2 * rng.random(162))
    mat["rho"] = mat["rho"] * (1 + 0.2 * rng.random(162))
    S = _solver(mat=mat, dt=5e-4)
    U = _random_smooth(S, 4)
    w = S.mesh.detJ
    tot0 = torch.einsum("m,mp->p", w, U[:, 0, :])
    D, _ = S.predict(U)
    Uz = S.time_points(D)
    _, src = S.volume_and_source(Uz)
    U1 = S.step(U)
    tot1 = torch.einsum("m,mp->p", w, U1[:, 0, :])
    scale = torch.einsum("m,mp->p", w, U[:, 0, :].abs())
    assert ((tot1[:9] - tot0[:9]).abs() <= 1e-13 * scale[:9] + 1e-30).all()
    dalpha = float(torch.einsum("m,m->", w, src[:, 0, 9]))
    assert dalpha > 0
    assert abs(float(tot1[9] - tot0[9]) - dalpha) < 1e-12 * float(scale[9])


def test_energy_does_not_increase_with_damage():
    from oracle.diagnostics import energy
    w = make_workload("c2", n=3, periodic=True)
    S = from_workload(w)
    U = S.project(w.ic)
    E0 = energy(S, U)
    for _ in range(3):
        U1 = S.step(U)
        E1 = energy(S, U1)
        assert E1 <= E0 * (1 + 1e-12)
        U, E0 = U1, E1
    assert float(U[:, 0, 9].sum()) > 0


def _plane_error(N, nsteps, n=3):
    w = make_workload("c1", n=n, N=N)
    S = from_workload(w)
    dt = make_workload("c1", n=n, N=3).dt
    S.dt = dt
    U = S.run(S.project(w.ic), nsteps)
    T = nsteps * dt
    ic = plane_wave_ic(1000.0, 1e-6, w.extra["cp"])
    Ue = S.project(lambda x, e: ic(x - np.array([w.extra["cp"] * T, 0, 0]), e))
    return float(torch.linalg.norm(U - Ue) / torch.linalg.norm(Ue))


def test_plane_wave_p_convergence():
    errs = [_plane_error(N, 6) for N in (1, 2, 3)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3


def test_plane_wave_h_convergence():
    e3 = _plane_error(2, 3, n=3)
    e6 = _plane_error(2, 3, n=6)
    assert e6 < e3 / 4.0          # better than second order already on this coarse pair


def test_face_points_shared_by_both_sides():
    w = make_workload("c1", n=3)
    S = from_workload(w)
    m, ref = S.mesh, S.ref
    ell = 1000.0
    for e in range(S.E):
        for f in range(4):
            mp, fp = int(m.nbr[e, f]), int(m.nbr_face[e, f])
            x = m.X0[e] + m.xiface[e, f] @ m.J[e].T
            xp = m.X0[mp] + m.xiface[mp, fp] @ m.J[mp].T
            d = (x - xp) / ell
            assert torch.allclose(d, torch.round(d), atol=1e-12)
            # points lie on the element's own face f
            xi = m.xiface[e, f]
            if f < 3:
                assert torch.allclose(xi[:, 2 - f], torch.zeros(ref.Ns, dtype=DT), atol=1e-15)
            else:
                assert torch.allclose(xi.sum(1), torch.ones(ref.Ns, dtype=DT))
            assert torch.allclose(ref.basis.values(m.xiface[mp, fp]), m.Fnbr[e, f])
            # opposite outward normals
            assert torch.allclose(m.normal[e, f], -m.normal[mp, fp], atol=1e-14)


# ---------------------------------------------------------------- brute force
def _rule(n):
    """Own Stroud rule (plain lists) with n points per direction."""
    ta, wa = roots_jacobi(n, 0, 0)
    tb, wb = roots_jacobi(n, 1, 0)
    tc, wc = roots_jacobi(n, 2, 0)
    pts = []
    for a, x in zip(ta, wa):
        for b, y in zip(tb, wb):
            for c, z in zip(tc, wc):
                pts.append(((1 + a) * (1 - b) * (1 - c) / 8, (1 + b) * (1 - c) / 4, (1 + c) / 2,
                            x * y * z / 64))
    return pts


def _tri_rule(n):
    ta, wa = roots_jacobi(n, 0, 0)
    tb, wb = roots_jacobi(n, 1, 0)
    return [((1 + a) * (1 - b) / 4, (1 + b) / 2, x * y / 4) for a, x in zip(ta, wa)
            for b, y in zip(tb, wb)]


@pytest.mark.parametrize("elastic", [True, False])
def test_single_element_brute_force(elastic):
    N = 2
    mat = _homog(162, Cd=0.0 if elastic else 1e-2)
    S = _solver(N=N, mat=mat, dt=4e-4)
    U = _random_smooth(S, 7)
    if elastic:
        U[..., 9] = 0.0
    e = 11
    ref, m = S.ref, S.mesh
    bas = ref.basis
    mloc = {k: v[e] for k, v in S.mat.items()}
    Jinv = m.Jinv[e].numpy()
    L = ref.L
    am = S.alpha_max

    def u_at(Ue, xi):
        return (bas.values(torch.tensor(xi, dtype=DT)[None]) @ Ue)[0]

    def grad_phys(xi):
        g = bas.gradients(torch.tensor(xi, dtype=DT)[None])[0].numpy()   # (3, L) d/dxi
        return Jinv.T @ g                                               # d/dx_d

    # (1) predictor: D^1_k = -int phi_k Bbar^d du/dx_d + int phi_k s(u)   (M = I)
    D, _ = S.predict(U)
    pts = _rule(N + 4)
    Bsum = np.zeros((3, 10, 10))
    wsum = 0.0
    for (x, y, z, wq) in _rule(N + 1):
        uq = u_at(U[e], (x, y, z))
        Bsum += wq * cdm.flux_jacobian(uq[None], mloc, am)[0].numpy()
        wsum += wq
    Bbar = Bsum / wsum
    D1 = np.zeros((L, 10))
    for (x, y, z, wq) in pts:
        xi = (x, y, z)
        phi = bas.values(torch.tensor(xi, dtype=DT)[None])[0].numpy()
        du = grad_phys(xi) @ U[e].numpy()                                # (3, 10)
        rhs = -sum(Bbar[d] @ du[d] for d in range(3))
        D1 += wq * np.outer(phi, rhs)
    for (x, y, z, wq) in _rule(N + 1):      # source on the nodal points, as in the paper
        phi = bas.values(torch.tensor((x, y, z), dtype=DT)[None])[0].numpy()
        uq = u_at(U[e], (x, y, z))
        D1[:, 9] += wq * phi * float(cdm.r_alpha(uq[None], mloc, am)[0])
    assert np.allclose(D[1][e].numpy(), D1, rtol=1e-11, atol=1e-11 * np.abs(D1).max())

    # (2) volume integral int dphi_k/dx_d F^d(u(t)) over space-time
    Uz = S.time_points(D)
    vol, _ = S.volume_and_source(Uz)
    V2 = np.zeros((L, 10))
    for z, gz in enumerate(ref.gamma.tolist()):
        for (x, y, zz, wq) in pts:
            xi = (x, y, zz)
            F = cdm.flux(u_at(Uz[z][e], xi)[None], mloc, am)[0].numpy()    # (3, 10)
            gp = grad_phys(xi)                                              # (3, L)
            V2 += S.dt * gz * wq * sum(np.outer(gp[d], F[d]) for d in range(3))
    tol = 1e-12 if elastic else 2e-2   # CDM flux is not polynomial: quadrature error only
    assert np.allclose(vol[e].numpy(), V2, rtol=0, atol=tol * np.abs(V2).max())

    # (3) face integral with a high-order face rule for face f
    f = 2
    face = S.face_term(Uz)
    mp, fp = int(m.nbr[e, f]), int(m.nbr_face[e, f])
    mlp = {k: v[mp] for k, v in S.mat.items()}
    n = m.normal[e, f]
    F2 = np.zeros((L, 10))
    for (h1, h2, bw) in _tri_rule(N + 4):
        bary = [1 - h1 - h2, h1, h2]
        nbb = [0.0, 0.0, 0.0]
        for j in range(3):
            nbb[m.slot_map[e, f, j]] = bary[j]
        xi_m = face_to_ref(f, torch.tensor([h1, h2], dtype=DT)).tolist()
        xi_p = face_to_ref(fp, torch.tensor(nbb[1:], dtype=DT)).tolist()
        phi = bas.values(torch.tensor(xi_m, dtype=DT)[None])[0].numpy()
        for z, gz in enumerate(ref.gamma.tolist()):
            uM = u_at(Uz[z][e], xi_m)
            uP = u_at(Uz[z][mp], xi_p)
            FM = torch.einsum("d,dp->p", n, cdm.flux(uM[None], mloc, am)[0])
            FP = torch.einsum("d,dp->p", n, cdm.flux(uP[None], mlp, am)[0])
            ub = 0.5 * (uM + uP)
            C = max(float(cdm.llf_speed(ub[None], n[None], mloc, am)[0]),
                    float(cdm.llf_speed(ub[None], n[None], mlp, am)[0]))
            Fs = (0.5 * (FM + FP) + 0.5 * C * (uM - uP)).numpy()
            F2 += S.dt * gz * bw * float(m.area[e, f] / m.detJ[e]) * np.outer(phi, Fs)
    single = torch.einsum("i,ik,ip->kp", ref.beta, m.Fface[e, f],
                          S.face_fluxes(Uz)[e, f]) * float(S.dt * m.area[e, f] / m.detJ[e])
    assert np.allclose(single.numpy(), F2, rtol=0, atol=(1e-12 if elastic else 2e-2) * np.abs(F2).max())
