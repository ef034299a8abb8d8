"""Stable Neo-Hookean energy density (oracle; test infrastructure only).

The paper uses "the Stable Neo-Hookean model" for 3D solids (Sec. 5.1,
Boundary conditions and materials) without printing its formula.  Reading
adopted here: the polynomial form

    psi(F) = mu/2 (tr(F^T F) - 3) - mu (J - 1) + lam/2 (J - 1)^2,   J = det F,

with (mu, lam) mapped from the Lame parameters (mu_L, lam_L) of (E, nu) as
mu = mu_L and lam = lam_L + mu_L, so that the tangent at F = I is the
isotropic linear-elasticity tensor of (mu_L, lam_L).

Vectorisation convention: vec(F) stacks the columns of F, so entry F[i, j]
sits at vec index 3*j + i.  All functions broadcast over leading axes.
"""
import numpy as np


def lame_to_snh(E, nu):
    """(mu, lam) of the energy above from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu_l = E / (2.0 * (1.0 + nu))
    lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu_l, lam_l + mu_l


def cofactor(F):
    """cof F = dJ/dF; its columns are f1 x f2, f2 x f0, f0 x f1 (f_j = columns of F)."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    return np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=-1)


def psi(F, mu, lam):
    """Energy density psi(F)."""
    J = np.linalg.det(F)
    Ic = np.sum(F * F, axis=(-2, -1))
    return 0.5 * mu * (Ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def first_piola(F, mu, lam):
    """P = dpsi/dF = mu F - mu cof F + lam (J - 1) cof F."""
    J = np.linalg.det(F)[..., None, None]
    C = cofactor(F)
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
    return mu * F - mu * C + lam * (J - 1.0) * C


def _cross_matrix(v):
    """[v]_x with [v]_x w = v x w."""
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], axis=-1),
        np.stack([v[..., 2], z, -v[..., 0]], axis=-1),
        np.stack([-v[..., 1], v[..., 0], z], axis=-1),
    ], axis=-2)


def hessian_of_det(F):
    """d^2 J / d vec(F)^2 (9x9).

    Block (j, l) is d(cof F column j)/d(column l of F):
      [[0, -[f2]x, [f1]x], [[f2]x, 0, -[f0]x], [-[f1]x, [f0]x, 0]].
    """
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    X0, X1, X2 = _cross_matrix(f0), _cross_matrix(f1), _cross_matrix(f2)
    Z = np.zeros_like(X0)
    rows = [
        np.concatenate([Z, -X2, X1], axis=-1),
        np.concatenate([X2, Z, -X0], axis=-1),
        np.concatenate([-X1, X0, Z], axis=-1),
    ]
    return np.concatenate(rows, axis=-2)


def vec(M):
    """Column-stacking vec of (..., 3, 3) -> (..., 9)."""
    return np.swapaxes(M, -1, -2).reshape(M.shape[:-2] + (9,))


def d2psi_dF2(F, mu, lam):
    """A = d^2 psi / d vec(F)^2 = mu I_9 + lam vec(cof F) vec(cof F)^T + (lam (J-1) - mu) d^2J/dF^2."""
    J = np.linalg.det(F)
    c = vec(cofactor(F))
    mu = np.asarray(mu, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    s = lam * (J - 1.0) - mu
    A = (mu[..., None, None] * np.eye(9)
         + lam[..., None, None] * c[..., :, None] * c[..., None, :]
         + s[..., None, None] * hessian_of_det(F))
    return A
