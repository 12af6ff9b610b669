"""Free-surface and absorbing boundary fluxes (oracle), Appendix A.3.

On domain boundaries only the isotropic part of the CDM Jacobian is kept: the
effective matrices B^{d,eff} in effective Lame parameters (Eqs. matrix_Beff_1..3,
effective-cdb; for the IVM law the caller passes Eq. effective-ivm).  The paper's
printed matrices carry typos; readings used here:

* the alpha row/column of B^{d,eff} is zero (alpha carries no flux; the
  printed 1 in entry (10,10) would contradict the zero eigenvalue of Lambda);
* c_s^eff = sqrt(mu_eff/rho) (printed as a second c_p^eff);
* row 2 of the stress matrix C is (lambda, lambda+2mu, lambda, 0, 0, 0) (the
  printed stray 1 in column 6 is dropped; that row is not used anyway);
* mu_eff = mu0 + alpha xi0 gamma_r - alpha gamma_r xi / 2, with the sign of
  the xi0 term taken from the stress law (Eq. cdb-model) where the appendix
  prints the opposite sign; lambda_eff = lambda0 - alpha gamma_r I1/(3 sqrt I2)
  as printed; both evaluated pointwise from the interior trace u^-.

Rotation T (Eq. matrix-T) takes face-aligned quantities (n, s, t frame) to the
global frame; T^{-1} is obtained with a linear solve.  Absorbing flux
(Eq. absorbing-flux): T R Lambda^+ R^{-1} T^{-1} u^-.  Free surface
(Eqs. q_b, matrix-C, freeSurface-flux): u^b = u' + sum_j omega_j r^j with the
three omegas solved so that sigma_nn = sigma_ns = sigma_nt = 0, then
F = T B^{1,eff} u^b.
"""
import torch

from .cdm import I2_MIN_F64, _parts

DT = torch.float64


def tangents(n):
    """s = normalise(n x e_k) for the axis e_k least aligned with n; t = n x s."""
    k = torch.argmin(torch.abs(n), dim=-1)
    e = torch.nn.functional.one_hot(k, 3).to(DT)
    s = torch.linalg.cross(n, e)
    s = s / torch.linalg.norm(s, dim=-1, keepdim=True)
    t = torch.linalg.cross(n, s)
    return s, t


def T_matrix(n, s, t):
    """Eq. matrix-T (rows xx, yy, zz, xy, yz, zx, vx, vy, vz, alpha)."""
    sh = n.shape[:-1]
    T = torch.zeros(*sh, 10, 10, dtype=DT)
    a = (n, s, t)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0))   # (i, j) of a row
    cols = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0))    # (a, b) of a column
    for r, (i, j) in enumerate(pairs):
        for c, (p, q) in enumerate(cols):
            if p == q:
                T[..., r, c] = a[p][..., i] * a[p][..., j]
            else:
                T[..., r, c] = a[p][..., i] * a[q][..., j] + a[q][..., i] * a[p][..., j]
    for i in range(3):
        for c in range(3):
            T[..., 6 + i, 6 + c] = a[c][..., i]
    T[..., 9, 9] = 1.0
    return T


def effective_lame(u, mat, alpha_max, i2_min=I2_MIN_F64):
    """lambda_eff, mu_eff of Eq. effective-cdb (readings in the module doc)."""
    I1, I2, s, xi, ac, _ = _parts(u, alpha_max, i2_min)
    lam = mat["lambda0"] - ac * mat["gamma_r"] * xi / 3.0
    mu = mat["mu0"] + ac * mat["xi0"] * mat["gamma_r"] - 0.5 * ac * mat["gamma_r"] * xi
    return lam, mu


def Beff1(lam, mu, rho):
    """B^{1,eff} (Eq. matrix_Beff_1) with the alpha entry set to zero."""
    B = torch.zeros(*lam.shape, 10, 10, dtype=DT)
    B[..., 0, 6] = -1.0
    B[..., 3, 7] = -0.5
    B[..., 5, 8] = -0.5
    B[..., 6, 0] = -(lam + 2 * mu) / rho
    B[..., 6, 1] = -lam / rho
    B[..., 6, 2] = -lam / rho
    B[..., 7, 3] = -2 * mu / rho
    B[..., 8, 5] = -2 * mu / rho
    return B


def R_matrix(lam, mu, rho):
    """Eigenvectors of B^{1,eff} (Eq. matrix-R), columns ordered like
    Lambda = diag(-cp, -cs, -cs, 0, 0, 0, cs, cs, cp, 0)."""
    cp = torch.sqrt((lam + 2 * mu) / rho)
    cs = torch.sqrt(mu / rho)
    r = lam / (lam + 2 * mu)
    R = torch.zeros(*lam.shape, 10, 10, dtype=DT)
    R[..., 0, 0] = 1.0
    R[..., 0, 3] = -r
    R[..., 0, 5] = -r
    R[..., 0, 8] = -1.0
    R[..., 1, 5] = 1.0
    R[..., 2, 3] = 1.0
    R[..., 3, 1] = 0.5
    R[..., 3, 7] = -0.5
    R[..., 4, 4] = 1.0
    R[..., 5, 2] = 0.5
    R[..., 5, 6] = -0.5
    R[..., 6, 0] = cp
    R[..., 6, 8] = cp
    R[..., 7, 1] = cs
    R[..., 7, 7] = cs
    R[..., 8, 2] = cs
    R[..., 8, 6] = cs
    R[..., 9, 9] = 1.0
    lam_diag = torch.stack([-cp, -cs, -cs, 0 * cp, 0 * cp, 0 * cp, cs, cs, cp, 0 * cp], -1)
    return R, lam_diag


def C_matrix(lam, mu):
    """Face-aligned strain -> stress map (Eq. matrix-C), row 2 as read above."""
    C = torch.zeros(*lam.shape, 10, 10, dtype=DT)
    for i in range(3):
        for j in range(3):
            C[..., i, j] = lam + (2 * mu if i == j else 0.0)
    for i in range(3, 6):
        C[..., i, i] = 2 * mu
    for i in range(6, 10):
        C[..., i, i] = 1.0
    return C


def _frame(u, n):
    s, t = tangents(n)
    T = T_matrix(n, s, t)
    up = torch.linalg.solve(T, u[..., None])[..., 0]          # T^{-1} u
    return T, up


def absorbing_flux(u, n, mat, alpha_max, i2_min=I2_MIN_F64, lame=None):
    """lame: the rheology's effective Lame parameters (default: CDM)."""
    lam, mu = (lame or effective_lame)(u, mat, alpha_max, i2_min)
    T, up = _frame(u, n)
    R, ld = R_matrix(lam, mu, mat["rho"])
    lplus = torch.clamp(ld, min=0.0)
    w = torch.linalg.solve(R, up[..., None])[..., 0]          # R^{-1} u'
    fp = (R @ (lplus * w)[..., None])[..., 0]
    return (T @ fp[..., None])[..., 0]


def free_surface_flux(u, n, mat, alpha_max, i2_min=I2_MIN_F64, lame=None):
    """lame: the rheology's effective Lame parameters (default: CDM)."""
    lam, mu = (lame or effective_lame)(u, mat, alpha_max, i2_min)
    T, up = _frame(u, n)
    R, _ = R_matrix(lam, mu, mat["rho"])
    C = C_matrix(lam, mu)
    rows = [0, 3, 5]                                          # sigma_nn, sigma_ns, sigma_tn
    rj = R[..., :, 0:3]                                       # r^1, r^2, r^3
    A = (C @ rj)[..., rows, :]                                # (..., 3, 3)
    b = -(C @ up[..., None])[..., rows, 0]
    omega = torch.linalg.solve(A, b[..., None])[..., 0]
    ub = up + (rj @ omega[..., None])[..., 0]
    B1 = Beff1(lam, mu, mat["rho"])
    return (T @ (B1 @ ub[..., None]))[..., 0]
