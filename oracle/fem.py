"""Linear tetrahedra, element quantities and the incremental potential (oracle; test infrastructure only).

Element e = (i0, i1, i2, i3) with rest shape matrix Dm = [X1-X0, X2-X0, X3-X0]
and rest volume V_e = det(Dm)/6 (must be > 0).  With b_1..b_3 the rows of
Dm^-1 and b_0 = -(b_1 + b_2 + b_3), the deformation gradient is
F = sum_a x_a b_a^T.  The linear map vec(F) = B_e x_e (x_e = [x0; x1; x2; x3],
12 entries, vertex-major) has B_e[3j+i, 3a+i] = b_a[j].

Element quantities by the chain rule (Sec. 3: element contributions that are
summed into H and g):
    psi_e = V_e psi(F),  g^e = V_e B_e^T vec(P(F)),  H^e = V_e B_e^T A(F) B_e.

Backward Euler as a minimisation (Sec. 5.1, time stepping; reading for the
terms the paper does not print):
    Psi(x) = sum_i m_i/(2h^2) |x_i - xhat_i|^2 + sum_e psi_e(x)
             + sum_{i in D} k_D/2 |x_i - xbar_i|^2,
    xhat = x^n + h v^n + h^2 g_grav,
with lumped masses m_i = sum_{e containing i} rho V_e / 4 and Dirichlet
constraints as penalty potentials (Sec. 5.1, boundary conditions).
"""
from dataclasses import dataclass

import numpy as np

from .snh import d2psi_dF2, first_piola, lame_to_snh, psi, vec

CHUNK = 65536  # elements per batch: bounds memory only, every element is independent


@dataclass
class Mesh:
    """Rest-state data of a tetrahedral mesh."""
    X: np.ndarray      # (N,3)
    tets: np.ndarray   # (T,4) int
    Bm: np.ndarray     # (T,3,3) = Dm^-1
    V: np.ndarray      # (T,)
    mu: np.ndarray     # (T,)
    lam: np.ndarray    # (T,)

    @classmethod
    def build(cls, X, tets, E, nu):
        X = np.asarray(X, dtype=np.float64)
        tets = np.asarray(tets, dtype=np.int64)
        if tets.min() < 0 or tets.max() >= X.shape[0]:
            raise ValueError("tet index out of range")
        Dm = np.stack([X[tets[:, a]] - X[tets[:, 0]] for a in (1, 2, 3)], axis=-1)
        detD = np.linalg.det(Dm)
        if np.any(detD <= 0.0):
            raise ValueError("degenerate or inverted rest tetrahedron")
        mu, lam = lame_to_snh(np.broadcast_to(E, tets.shape[:1]), np.broadcast_to(nu, tets.shape[:1]))
        return cls(X=X, tets=tets, Bm=np.linalg.inv(Dm), V=detD / 6.0, mu=mu, lam=lam)

    @property
    def n_verts(self):
        return self.X.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]

    def shape_vectors(self, sel=slice(None)):
        """b_a for a = 0..3 as (T,4,3)."""
        Bm = self.Bm[sel]
        b123 = Bm  # rows of Dm^-1
        b0 = -(b123[:, 0] + b123[:, 1] + b123[:, 2])
        return np.concatenate([b0[:, None, :], b123], axis=1)

    def B_matrix(self, sel=slice(None)):
        """B_e (T,9,12) with vec(F) = B_e x_e."""
        b = self.shape_vectors(sel)
        T = b.shape[0]
        B = np.zeros((T, 9, 12))
        for a in range(4):
            for i in range(3):
                for j in range(3):
                    B[:, 3 * j + i, 3 * a + i] = b[:, a, j]
        return B

    def deformation_gradient(self, x, sel=slice(None)):
        """F = sum_a x_a b_a^T as (T,3,3)."""
        b = self.shape_vectors(sel)
        xe = x[self.tets[sel]]  # (T,4,3)
        return np.einsum("tai,taj->tij", xe, b)


def lumped_mass(mesh: Mesh, rho):
    """m_i = sum over elements containing i of rho V_e / 4."""
    m = np.zeros(mesh.n_verts)
    for a in range(4):
        np.add.at(m, mesh.tets[:, a], rho * mesh.V / 4.0)
    return m


def element_psi(mesh: Mesh, x):
    """psi_e = V_e psi(F_e) for all elements, (T,)."""
    out = np.empty(mesh.n_tets)
    for s in range(0, mesh.n_tets, CHUNK):
        sel = slice(s, min(mesh.n_tets, s + CHUNK))
        F = mesh.deformation_gradient(x, sel)
        out[sel] = mesh.V[sel] * psi(F, mesh.mu[sel], mesh.lam[sel])
    return out


def element_grad(mesh: Mesh, x):
    """g^e (T,12) for all elements (the gradient half of ``element_grad_hess``)."""
    g = np.empty((mesh.n_tets, 12))
    for s in range(0, mesh.n_tets, CHUNK):
        sel = slice(s, min(mesh.n_tets, s + CHUNK))
        F = mesh.deformation_gradient(x, sel)
        B = mesh.B_matrix(sel)
        P = first_piola(F, mesh.mu[sel], mesh.lam[sel])
        g[sel] = mesh.V[sel][:, None] * np.einsum("tki,tk->ti", B, vec(P))
    return g


def element_grad_hess(mesh: Mesh, x, idx=None):
    """(g^e (n,12), H^e (n,12,12)), unprojected, for the elements ``idx`` (all if None)."""
    idx = np.arange(mesh.n_tets) if idx is None else np.asarray(idx, dtype=np.int64)
    g = np.empty((idx.size, 12))
    H = np.empty((idx.size, 12, 12))
    for s in range(0, idx.size, CHUNK):
        sel = idx[s:s + CHUNK]
        loc = slice(s, s + sel.size)
        F = mesh.deformation_gradient(x, sel)
        B = mesh.B_matrix(sel)
        V = mesh.V[sel]
        P = first_piola(F, mesh.mu[sel], mesh.lam[sel])
        A = d2psi_dF2(F, mesh.mu[sel], mesh.lam[sel])
        g[loc] = V[:, None] * np.einsum("tki,tk->ti", B, vec(P))
        H[loc] = V[:, None, None] * np.matmul(np.swapaxes(B, 1, 2), np.matmul(A, B))
    return g, H


def predictor(x_n, v_n, h, gravity):
    """xhat = x^n + h v^n + h^2 g_grav."""
    return x_n + h * v_n + h * h * np.asarray(gravity, dtype=np.float64)[None, :]
