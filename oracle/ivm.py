"""Pointwise internal-variable-model (IVM) rheology (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Same state vector and conservation form as the CDM law (oracle.cdm); the
constitutive law of Section 2.1, Eq. ivm-model, with the Murnaghan terms
switched off (l0 = m0 = n0 = 0, as the paper does for its algorithm):
    sigma = (1 - alpha) (lambda0 I1 delta + 2 mu0 eps)
    r_alpha = [lambda0 I1^2 / 2 + mu0 I2 - phi(alpha)] / (gamma_b tau_b),
    phi(alpha) = gamma_b (alpha / (1 - alpha))^2
with I1 = eps_kk, I2 = eps_ij eps_ij (both shear entries counted).

Reading: alpha is clamped to [0, alpha_max] wherever it is used, as for the
CDM law (the storage energy phi is singular at alpha = 1); the stored modal
alpha is never modified.  The law is smooth, so no invariant guard is needed.
Effective Lame parameters on boundaries (Eq. effective-ivm):
(1 - alpha) lambda0, (1 - alpha) mu0.
"""
import torch
from torch.func import jacfwd, vmap

from .cdm import DT, I2_MIN_F64, flux_of_stress, invariants

MAT_KEYS = ("rho", "lambda0", "mu0", "gamma_b", "tau_b")


def _ac(u, alpha_max):
    return torch.clamp(u[..., 9], 0.0, alpha_max)


def stress(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """sigma (..., 6) in the order xx, yy, zz, xy, yz, zx (Eq. ivm-model)."""
    I1, _ = invariants(u)
    g = 1.0 - _ac(u, alpha_max)
    sig = (2.0 * mat["mu0"] * g)[..., None] * u[..., :6]
    iso = mat["lambda0"] * g * I1
    return sig + torch.cat([iso[..., None].expand(*iso.shape, 3),
                            torch.zeros(*iso.shape, 3, dtype=u.dtype)], -1)


def r_alpha(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """Damage rate of Eq. ivm-model (negative when phi exceeds the strain energy)."""
    I1, I2 = invariants(u)
    ac = _ac(u, alpha_max)
    phi = mat["gamma_b"] * (ac / (1.0 - ac)) ** 2
    return (0.5 * mat["lambda0"] * I1 * I1 + mat["mu0"] * I2 - phi) / (mat["gamma_b"] * mat["tau_b"])


def flux(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """F^d_p (..., 3, 10), Eq. nonlinear hyper pdes with the IVM stress."""
    return flux_of_stress(stress(u, mat, alpha_max), u, mat["rho"])


def _flux_point(u, rho, lam, mu, gb, tb, alpha_max, i2_min):
    mat = dict(rho=rho, lambda0=lam, mu0=mu, gamma_b=gb, tau_b=tb)
    return flux(u, mat, alpha_max, i2_min)


def flux_jacobian(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """B^d_pq = dF^d_p / du_q  (..., 3, 10, 10) by automatic differentiation."""
    shape = u.shape[:-1]
    uf = u.reshape(-1, 10)
    ms = [torch.broadcast_to(torch.as_tensor(mat[k], dtype=DT), shape).reshape(-1)
          for k in MAT_KEYS]
    jac = vmap(jacfwd(_flux_point, argnums=0),
               in_dims=(0, 0, 0, 0, 0, 0, None, None))(uf, *ms, alpha_max, i2_min)
    return jac.reshape(*shape, 3, 10, 10)


def normal_jacobian(u, n, mat, alpha_max, i2_min=I2_MIN_F64):
    """B_n = sum_d n_d B^d at states u (..., 10), normals n (..., 3)."""
    return torch.einsum("...d,...dpq->...pq", n, flux_jacobian(u, mat, alpha_max, i2_min))


def llf_speed(u, n, mat, alpha_max, i2_min=I2_MIN_F64):
    """Largest eigenvalue (real part) of B_n(u) (Eq. rusanov-flux)."""
    ev = torch.linalg.eigvals(normal_jacobian(u, n, mat, alpha_max, i2_min))
    return ev.real.max(dim=-1).values


def effective_lame(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """lambda_eff, mu_eff of Eq. effective-ivm."""
    g = 1.0 - _ac(u, alpha_max)
    return g * mat["lambda0"], g * mat["mu0"]
