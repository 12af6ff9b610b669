"""The five synthetic workloads (seeded) and their smaller cuts.

Every workload is a cube mesh from :mod:`workloads.mesh` plus per-element
materials, an initial-condition function, a fixed time step, optional point
sources and receivers.  Nothing here discretises the PDE.

Workload recipe (seeds: 0 initial condition and material, 1 source,
2 observed-model perturbation):

* ``c1`` periodic [0,1000 m]^3, 4^3 cubes x 6 = 384 tets, N=2, homogeneous
  rho=2700, lambda=mu=3.24e10 Pa, gamma_r=37 GPa, xi0=-0.75, C_d=0 (the
  damage parameters of the paper's anisotropy verification table); planar P
  wave along x with strain amplitude 1e-6, alpha=0; 100 steps at CFL 0.5.
* ``c2`` [0,1000 m]^3, 48^3 cubes, N=3, free top / absorbing sides; soft basin
  z >= 900 m (vs 400, vp 1200, rho 1900) over rock (vs 6000/sqrt3, vp 6000,
  rho 2700); gamma_r = (37/32) mu0, xi0 = -0.75, C_d = 1e8 s^-1 / gamma_r;
  initial strain = 32 Gaussian pulses (width 50 m, amplitude U(0,1e-4),
  random symmetric direction of unit Frobenius norm), v = 0, alpha0 per
  element U(0, 0.05); 500 steps.
* ``c3`` as c2 with 64^3 cubes, N=4 and a lognormal (sigma 10 %, Gaussian
  correlation 200 m) perturbation of mu0 and lambda0; 1000 steps.
* ``c4`` [0,24 km]^3, 24^3 cubes, N=3, c2's layered medium scaled to the box,
  a 2 Hz Ricker moment-rate point source 3 km below the free surface with random double-couple
  orientation, 16 receivers near the top face; 400 steps.
* ``c5`` [0,24 km]^3, 96^3 cubes, N=4, a 3 km basin whose vs rises linearly
  from 300 m/s at the surface to 2000 m/s, 64 subfault point sources on a
  30-degree dipping plane; 2000 steps.
* ``c5f`` c5 on a mesh graded in depth: 16 of the 96 layers, 8 times thinner
  than the others, form a band centred on the fault (6 km deep), as a mesh
  refined around a fault would; its global step is that band's (the
  workload for local time stepping).

``rheology="ivm"`` keeps any recipe's mesh, elastic model, initial condition
and sources and gives the IVM law its parameters: gamma_b = 0.5 kPa in
sediments (c_s < 1000 m/s) and 356 kPa in rock (Table 2's basin and upper
crust), tau_b = 1e-4 s.

Points placed on mesh faces would make the host element search ambiguous,
so receivers and the c4 source are nudged off the structured grid planes.
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .mesh import cube_mesh, kuhn_inradius, tet_inradius

ALPHA_MAX = 0.5
CFL = 0.5
# IVM damage time scale: the paper's 10 s shortened so that damage evolves
# (grows in strained rock, heals where the storage energy exceeds the strain
# energy) within runs of tens of steps
TAU_B_IVM = 1e-4

STF_RICKER = 0
STF_GAUSSIAN = 1


def table1_material():
    """CDM parameters of the paper's anisotropy verification (Table 1)."""
    return dict(rho=2760.0, lambda0=32e9, mu0=32e9, gamma_r=37e9, xi0=-0.75,
                Cd=0.0)


@dataclass
class Workload:
    name: str
    N: int
    mesh: dict
    material: dict            # per-element arrays rho, lambda0, mu0, gamma_r, xi0, Cd
    dt: float
    nsteps: int
    ic: Callable              # ic(x (npts,3), elem (npts,)) -> (npts, 10)
    alpha_max: float = ALPHA_MAX
    sources: Optional[dict] = None   # xyz (n,3), M6 (n,6), t_onset (n,), stf_param (n,), stf_kind
    receivers: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)
    rheology: str = "cdm"     # "cdm" (Eq. cdb-model) or "ivm" (Eq. ivm-model)

    @property
    def ne(self):
        return int(self.mesh["tets"].shape[0])

    @property
    def L(self):
        return (self.N + 1) * (self.N + 2) * (self.N + 3) // 6


def cfl_dt(mesh, material, N, cfl=CFL):
    """Global step from the intact moduli: cfl * 2 r_in / ((2N+1) c_p,max) on
    a uniform mesh; on a graded one the smallest cfl * 2 r_in,e / ((2N+1) c_p,e)
    over the elements."""
    cp = np.sqrt((material["lambda0"] + 2.0 * material["mu0"]) / material["rho"])
    if mesh.get("z_nodes") is None:
        r_in = kuhn_inradius(mesh["edge"])
        return cfl * 2.0 * r_in / ((2 * N + 1) * float(cp.max()))
    r = tet_inradius(mesh["xyz"], mesh["tets"])
    return cfl * 2.0 * float(np.min(r / cp)) / (2 * N + 1)


def fault_band_nodes(n, length, centre_depth=6000.0, factor=8):
    """Node heights of n layers: a band of max(1, n // 6) layers, `factor`
    times thinner than the others, centred `centre_depth` below the top (a
    mesh refined around a fault); the other layers share the rest equally."""
    m = max(1, n // 6)
    zc = length - centre_depth
    a = length / (n - m + m / factor)             # coarse spacing
    k1 = int(round((zc - 0.5 * m * a / factor) / a))
    k1 = min(max(k1, 0), n - m)
    k2 = n - m - k1
    a = length / (k1 + k2 + m / factor)
    steps = [a] * k1 + [a / factor] * m + [a] * k2
    z = np.concatenate([[0.0], np.cumsum(steps)])
    z[-1] = length
    return z


def _centroids(mesh):
    return mesh["xyz"][mesh["tets"]].mean(axis=1)


def _homogeneous(ne, rho, lam, mu, gamma_r, xi0, Cd):
    f = lambda v: np.full(ne, float(v))
    return dict(rho=f(rho), lambda0=f(lam), mu0=f(mu), gamma_r=f(gamma_r),
                xi0=f(xi0), Cd=f(Cd))


def _layered(mesh, basin_frac=0.1, c_d=1e8):
    """Soft basin in the top ``basin_frac`` of the box over rock."""
    c = _centroids(mesh)
    zt = mesh["xyz"][:, 2].max()
    ell = mesh["length"]
    basin = c[:, 2] >= zt - basin_frac * ell
    vs = np.where(basin, 400.0, 6000.0 / math.sqrt(3.0))
    vp = np.where(basin, 1200.0, 6000.0)
    rho = np.where(basin, 1900.0, 2700.0)
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    gamma_r = (37.0 / 32.0) * mu
    return dict(rho=rho, lambda0=lam, mu0=mu, gamma_r=gamma_r,
                xi0=np.full_like(mu, -0.75), Cd=c_d / gamma_r)


def _gradient_basin(mesh, depth=3000.0, c_d=1e8):
    """Basin of ``depth`` below the top with vs rising linearly 300 -> 2000."""
    c = _centroids(mesh)
    zt = mesh["xyz"][:, 2].max()
    d = zt - c[:, 2]
    basin = d <= depth
    vs_b = 300.0 + (2000.0 - 300.0) * np.clip(d / depth, 0.0, 1.0)
    vs = np.where(basin, vs_b, 6000.0 / math.sqrt(3.0))
    vp = np.where(basin, 3.0 * vs_b, 6000.0)
    rho = np.where(basin, 1900.0, 2700.0)
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    gamma_r = (37.0 / 32.0) * mu
    return dict(rho=rho, lambda0=lam, mu0=mu, gamma_r=gamma_r,
                xi0=np.full_like(mu, -0.75), Cd=c_d / gamma_r)


def _lognormal(mesh, rng, sigma=0.1, corr=200.0):
    """Unit-variance Gaussian random field on the cube grid (FFT synthesis,
    Gaussian covariance exp(-r^2/corr^2)), one value per cube."""
    n = mesh["n"]
    h = mesh["edge"]
    w = rng.standard_normal((n, n, n))
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=h)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    amp = np.exp(-(kx**2 + ky**2 + kz**2) * corr**2 / 8.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    g = (g - g.mean()) / g.std()
    # element e lives in cube e // 6 whose index is i + n*(j + n*k)
    gk = g.transpose(2, 1, 0).ravel()     # index [k][j][i] -> i fastest
    return np.exp(sigma * gk - 0.5 * sigma * sigma)


def plane_wave_ic(length, amplitude, cp):
    """Right-going P wave along x: eps_xx = A sin(2 pi x / length),
    v_x = -cp eps_xx, everything else zero."""
    def ic(x, elem=None):
        out = np.zeros((x.shape[0], 10))
        s = amplitude * np.sin(2.0 * math.pi * x[:, 0] / length)
        out[:, 0] = s
        out[:, 6] = -cp * s
        return out
    return ic


def _pulses_ic(mesh, rng, alpha0, npulse=32, width=50.0, amax=1e-4):
    o = mesh["xyz"].min(axis=0)
    ell = mesh["length"]
    centres = o + ell * rng.random((npulse, 3))
    amps = amax * rng.random(npulse)
    dirs = rng.standard_normal((npulse, 6))
    fro = np.sqrt((dirs[:, :3]**2).sum(1) + 2.0 * (dirs[:, 3:]**2).sum(1))
    dirs = dirs / fro[:, None]

    def ic(x, elem):
        # pulse profiles (points x pulses), then one product with the directions
        xt = np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)
        g = np.empty((xt.shape[1], npulse))
        for k in range(npulse):
            r2 = (xt[0] - centres[k, 0])**2 + (xt[1] - centres[k, 1])**2 + (xt[2] - centres[k, 2])**2
            g[:, k] = amps[k] * np.exp(r2 * (-1.0 / (2.0 * width * width)))
        out = np.zeros((xt.shape[1], 10))
        out[:, :6] = g @ dirs
        out[:, 9] = alpha0[elem]
        return out
    return ic


def _zero_ic(alpha0):
    def ic(x, elem):
        out = np.zeros((x.shape[0], 10))
        out[:, 9] = alpha0[elem]
        return out
    return ic


def _double_couple(rng):
    nrm = rng.standard_normal(3)
    nrm /= np.linalg.norm(nrm)
    s = rng.standard_normal(3)
    s -= s.dot(nrm) * nrm
    s /= np.linalg.norm(s)
    m = np.outer(s, nrm) + np.outer(nrm, s)
    return np.array([m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[1, 2], m[2, 0]])


def _receivers_top(mesh, depth=1.0):
    o = mesh["xyz"].min(axis=0)
    ell = mesh["length"]
    fr = np.array([1, 3, 5, 7]) / 8.0
    pts = []
    for fy in fr:
        for fx in fr:
            pts.append([o[0] + fx * ell + 0.0371 * mesh["edge"],
                        o[1] + fy * ell + 0.0137 * mesh["edge"],
                        o[2] + ell - depth])
    return np.asarray(pts)


def _finite_fault(mesh, rng, mu_src):
    """8 x 8 subfaults of 1 km^2 on an 8 km x 8 km plane dipping 30 degrees,
    centred 6 km below the top; thrust slip (rake 90 deg), Gaussian STF."""
    o = mesh["xyz"].min(axis=0)
    ell = mesh["length"]
    centre = np.array([o[0] + ell / 2, o[1] + ell / 2, o[2] + ell - 6000.0])
    dip = math.radians(30.0)
    strike_dir = np.array([1.0, 0.0, 0.0])
    dip_dir = np.array([0.0, math.cos(dip), -math.sin(dip)])     # down-dip
    normal = np.cross(strike_dir, dip_dir)
    normal /= np.linalg.norm(normal)
    slip_dir = -dip_dir                                           # up-dip (thrust)
    m = np.outer(slip_dir, normal) + np.outer(normal, slip_dir)
    m6 = np.array([m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[1, 2], m[2, 0]])
    xs, M6, onset = [], [], []
    slip = 5.0 * rng.random((8, 8))
    hypo = centre + (rng.random() - 0.5) * 8000.0 * strike_dir \
        + (rng.random() - 0.5) * 8000.0 * dip_dir
    for a in range(8):
        for b in range(8):
            p = centre + (a - 3.5) * 1000.0 * strike_dir + (b - 3.5) * 1000.0 * dip_dir
            xs.append(p)
            M6.append(mu_src * 1e6 * slip[a, b] * m6)
            onset.append(np.linalg.norm(p - hypo) / 2800.0 + 0.1 * rng.random())
    n = len(xs)
    return dict(xyz=np.asarray(xs), M6=np.asarray(M6), t_onset=np.asarray(onset),
                stf_param=np.full(n, 0.1), stf_kind=STF_GAUSSIAN)


CONFIGS = {
    "c1": dict(n=4, length=1000.0, N=2, nsteps=100),
    "c2": dict(n=48, length=1000.0, N=3, nsteps=500),
    "c3": dict(n=64, length=1000.0, N=4, nsteps=1000),
    "c4": dict(n=24, length=24000.0, N=3, nsteps=400),
    "c5": dict(n=96, length=24000.0, N=4, nsteps=2000),
    # c5 on a mesh refined 8x in depth around the fault (for local time stepping)
    "c5f": dict(n=96, length=24000.0, N=4, nsteps=2000),
}


def ivm_material(material, tau_b=TAU_B_IVM):
    """IVM parameters on the same elastic model: rho, lambda0, mu0 kept,
    gamma_b = 0.5 kPa in sediments (c_s < 1000 m/s) and 356 kPa in rock (the
    basin and upper-crust units of Table 2), tau_b per element."""
    mu, rho = material["mu0"], material["rho"]
    soft = np.sqrt(mu / rho) < 1000.0
    gb = np.where(soft, 0.5e3, 356e3)
    return dict(rho=rho.copy(), lambda0=material["lambda0"].copy(), mu0=mu.copy(),
                gamma_b=gb, tau_b=np.full_like(mu, tau_b))


def make_workload(name, n=None, N=None, nsteps=None, seed=0, periodic=None, rheology="cdm"):
    """Build workload ``name`` (c1..c5); ``n``/``N``/``nsteps`` override the
    mesh resolution, polynomial degree and step count (smaller cuts of the
    same recipe); ``rheology="ivm"`` puts the IVM parameters (``ivm_material``)
    on the same elastic model, initial condition and sources."""
    wl = _make(name, n, N, nsteps, seed, periodic)
    if rheology == "ivm":
        wl.material = ivm_material(wl.material)
        wl.rheology = "ivm"
    elif rheology != "cdm":
        raise ValueError(f"unknown rheology {rheology!r}")
    return wl


def _make(name, n, N, nsteps, seed, periodic):
    cfg = dict(CONFIGS[name])
    n = cfg["n"] if n is None else int(n)
    N = cfg["N"] if N is None else int(N)
    nsteps = cfg["nsteps"] if nsteps is None else int(nsteps)
    ell = cfg["length"]
    rng = np.random.default_rng(seed)
    if name == "c1":
        mesh = cube_mesh(n, ell, periodic=True if periodic is None else periodic)
        ne = mesh["tets"].shape[0]
        mat = _homogeneous(ne, 2700.0, 3.24e10, 3.24e10, 37e9, -0.75, 0.0)
        cp = math.sqrt((3.24e10 + 2 * 3.24e10) / 2700.0)
        ic = plane_wave_ic(ell, 1e-6, cp)
        wl = Workload(name, N, mesh, mat, cfl_dt(mesh, mat, N), nsteps, ic)
        wl.extra["cp"] = cp
        wl.extra["amplitude"] = 1e-6
        return wl
    zn = fault_band_nodes(n, ell) if name == "c5f" else None
    mesh = cube_mesh(n, ell, periodic=bool(periodic), z_nodes=zn)
    ne = mesh["tets"].shape[0]
    if name in ("c2", "c3", "c4"):
        mat = _layered(mesh)
    else:
        mat = _gradient_basin(mesh)
    if name == "c3":
        f = _lognormal(mesh, rng)
        per_elem = np.repeat(f, 6)
        mat["mu0"] = mat["mu0"] * per_elem
        mat["lambda0"] = mat["lambda0"] * per_elem
        mat["gamma_r"] = (37.0 / 32.0) * mat["mu0"]
        mat["Cd"] = 1e8 / mat["gamma_r"]
    alpha0 = 0.05 * rng.random(ne)
    if name in ("c2", "c3"):
        ic = _pulses_ic(mesh, rng, alpha0)
    else:
        ic = _zero_ic(alpha0)
    wl = Workload(name, N, mesh, mat, cfl_dt(mesh, mat, N), nsteps, ic)
    wl.extra["alpha0"] = alpha0
    src_rng = np.random.default_rng(seed + 1)
    if name == "c4":
        o = mesh["xyz"].min(axis=0)
        # 3 km below the free surface (under the soft layer), so that the 400
        # steps (~2 s) record arrivals at the receivers near the surface
        xs = o + np.array([ell / 2 + 0.0113 * mesh["edge"],
                           ell / 2 + 0.0079 * mesh["edge"],
                           ell - 3000.0 - 0.0053 * mesh["edge"]])
        f0 = 2.0
        wl.sources = dict(xyz=xs[None, :], M6=1e15 * _double_couple(src_rng)[None, :],
                          t_onset=np.array([1.2 / f0]), stf_param=np.array([f0]),
                          stf_kind=STF_RICKER)
        wl.receivers = _receivers_top(mesh)
    if name in ("c5", "c5f"):
        wl.sources = _finite_fault(mesh, src_rng, 3.24e10)
        wl.receivers = _receivers_top(mesh)
    return wl


def perturbed_material(material, seed=2, rel_mu=0.05, rel_cd=0.2):
    """Observed-model material for the misfit: mu0 (1 + 0.05 g), C_d (1 + 0.2 g').
    gamma_r keeps its ratio 37/32 to mu0 in the perturbed model (as in every
    material of the recipes), so that the damaged moduli stay positive up to
    the clamp alpha_max; the gradient itself is taken with gamma_r fixed."""
    rng = np.random.default_rng(seed)
    ne = material["mu0"].shape[0]
    out = {k: v.copy() for k, v in material.items()}
    f = 1.0 + rel_mu * rng.standard_normal(ne)
    out["mu0"] = material["mu0"] * f
    if "gamma_r" in out:
        out["gamma_r"] = material["gamma_r"] * f
    out["Cd"] = material["Cd"] * (1.0 + rel_cd * rng.standard_normal(ne))
    return out
