"""Pointwise continuum-damage (CDM) rheology (oracle).

State vector (Section 2.1, Eq. nonlinear hyper pdes), tensor (not engineering)
shear strains:
    u = (eps_xx, eps_yy, eps_zz, eps_xy, eps_yz, eps_zx, v_x, v_y, v_z, alpha)

Constitutive law of Lyakhovsky et al. as written in Eq. cdb-model:
    sigma = lambda0 I1 delta - alpha gamma_r sqrt(I2) delta
            + [2 (mu0 + alpha xi0 gamma_r) - alpha gamma_r xi] eps
    r_alpha = C_d gamma_r I2 (xi - xi0)  if xi > xi0, else 0
with I1 = eps_kk, I2 = eps_ij eps_ij (both shear entries counted), xi = I1/sqrt(I2).

Readings where the paper is silent:
* alpha is clamped to [0, alpha_max] wherever it is used (the paper keeps
  alpha in [0, 1]); the stored modal alpha is never modified.
* for I2 <= I2_min the sqrt(I2) and xi terms are dropped (xi := 0,
  sqrt(I2) := 0) and r_alpha := 0, so that nothing divides by zero.

Conservation form (Eq. nonlinear hyper pdes): du/dt + dF^d/dx_d = s with
    F^d(eps_ij) = -(v_i delta_jd + v_j delta_id)/2,  F^d(v_i) = -sigma_id/rho,
    F^d(alpha) = 0,   s = (0, ..., 0, r_alpha).
The Jacobians B^d = dF^d/du (Eq. nonlinear-wave) are taken by automatic
differentiation of the flux (torch.func), i.e. straight from their definition.
The local Lax-Friedrichs constant C is the largest eigenvalue of
B_n = n_d B^d evaluated at the mean state (Eq. rusanov-flux), taken from a
general eigen-solver of the 10x10 matrix.
"""
import torch
from torch.func import jacfwd, vmap

DT = torch.float64
I2_MIN_F64 = 1e-30
# (i, j) of the six strain / stress components and the symmetric-index table
VOIGT = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0))
SYM = ((0, 3, 5), (3, 1, 4), (5, 4, 2))     # component index of (i, j)
MAT_KEYS = ("rho", "lambda0", "mu0", "gamma_r", "xi0", "Cd")


def invariants(u):
    e = u[..., :6]
    I1 = e[..., 0] + e[..., 1] + e[..., 2]
    I2 = (e[..., :3] ** 2).sum(-1) + 2.0 * (e[..., 3:6] ** 2).sum(-1)
    return I1, I2


def _parts(u, alpha_max, i2_min):
    I1, I2 = invariants(u)
    guard = I2 <= i2_min
    I2s = torch.where(guard, torch.ones_like(I2), I2)
    s = torch.where(guard, torch.zeros_like(I2), torch.sqrt(I2s))
    xi = torch.where(guard, torch.zeros_like(I2), I1 / torch.sqrt(I2s))
    ac = torch.clamp(u[..., 9], 0.0, alpha_max)
    return I1, I2, s, xi, ac, guard


def stress(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """sigma (..., 6) in the order xx, yy, zz, xy, yz, zx (Eq. cdb-model)."""
    I1, I2, s, xi, ac, _ = _parts(u, alpha_max, i2_min)
    lam, mu, gr, xi0 = mat["lambda0"], mat["mu0"], mat["gamma_r"], mat["xi0"]
    iso = lam * I1 - ac * gr * s
    coef = 2.0 * (mu + ac * xi0 * gr) - ac * gr * xi
    sig = coef[..., None] * u[..., :6]
    sig = sig + torch.cat([iso[..., None].expand(*iso.shape, 3),
                           torch.zeros(*iso.shape, 3, dtype=u.dtype)], -1)
    return sig


def r_alpha(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """Damage rate of Eq. cdb-model (zero below the threshold xi0)."""
    I1, I2, s, xi, ac, guard = _parts(u, alpha_max, i2_min)
    r = mat["Cd"] * mat["gamma_r"] * I2 * (xi - mat["xi0"])
    return torch.where(guard | (xi <= mat["xi0"]), torch.zeros_like(r), r)


def energy_density(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """W = lambda0 I1^2/2 + (mu0 + alpha xi0 gamma_r) I2 - alpha gamma_r I1 sqrt(I2),
    whose strain derivative is the stress of Eq. cdb-model."""
    I1, I2, s, xi, ac, _ = _parts(u, alpha_max, i2_min)
    return (0.5 * mat["lambda0"] * I1 * I1
            + (mat["mu0"] + ac * mat["xi0"] * mat["gamma_r"]) * I2
            - ac * mat["gamma_r"] * I1 * s)


def flux(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """F^d_p (..., 3, 10), Eq. nonlinear hyper pdes."""
    return flux_of_stress(stress(u, mat, alpha_max, i2_min), u, mat["rho"])


def flux_of_stress(sig, u, rho):
    """F^d_p (..., 3, 10) of Eq. nonlinear hyper pdes for a given stress (any
    rheology): strain rows from the velocity, velocity rows -sigma_id/rho."""
    v = u[..., 6:9]
    zero = torch.zeros_like(v[..., 0])
    rows = []
    for d in range(3):
        comp = []
        for (i, j) in VOIGT:
            val = zero
            if j == d:
                val = val - 0.5 * v[..., i]
            if i == d:
                val = val - 0.5 * v[..., j]
            comp.append(val)
        for i in range(3):
            comp.append(-sig[..., SYM[i][d]] / rho)
        comp.append(zero)
        rows.append(torch.stack(comp, dim=-1))
    return torch.stack(rows, dim=-2)


def _flux_point(u, rho, lam, mu, gr, xi0, cd, alpha_max, i2_min):
    mat = dict(rho=rho, lambda0=lam, mu0=mu, gamma_r=gr, xi0=xi0, Cd=cd)
    return flux(u, mat, alpha_max, i2_min)


def flux_jacobian(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """B^d_pq = dF^d_p / du_q  (..., 3, 10, 10) by automatic differentiation."""
    shape = u.shape[:-1]
    uf = u.reshape(-1, 10)
    ms = [torch.broadcast_to(torch.as_tensor(mat[k], dtype=DT), shape).reshape(-1)
          for k in MAT_KEYS]
    jac = vmap(jacfwd(_flux_point, argnums=0),
               in_dims=(0, 0, 0, 0, 0, 0, 0, None, None))(uf, *ms, alpha_max, i2_min)
    return jac.reshape(*shape, 3, 10, 10)


def normal_jacobian(u, n, mat, alpha_max, i2_min=I2_MIN_F64):
    """B_n = sum_d n_d B^d at states u (..., 10), normals n (..., 3)."""
    B = flux_jacobian(u, mat, alpha_max, i2_min)
    return torch.einsum("...d,...dpq->...pq", n, B)


def llf_speed(u, n, mat, alpha_max, i2_min=I2_MIN_F64):
    """Largest eigenvalue (real part) of B_n(u) (Eq. rusanov-flux)."""
    Bn = normal_jacobian(u, n, mat, alpha_max, i2_min)
    ev = torch.linalg.eigvals(Bn)
    return ev.real.max(dim=-1).values
