"""Global assembly of the incremental potential's gradient and Hessian
(oracle; test infrastructure only).

Sec. 3: H = sum_e H^e and g = sum_e g^e, where each element's 12 rows and
columns land on the 3 DOFs of each of its 4 vertices; the inertia and
Dirichlet-penalty terms add per-vertex diagonal contributions.  The sparse
sum is SciPy's COO -> CSR conversion, which adds duplicate entries.
Sec. 4.1: projecting element e changes H by Delta H^e = Hhat^e - H^e
(Eq. (5)) without changing its sparsity.
"""
import numpy as np
import scipy.sparse as sp


class Assembler:
    """Index maps from element-local 12x12 entries to global DOFs."""

    def __init__(self, tets, n_verts):
        tets = np.asarray(tets, dtype=np.int64)
        self.n = 3 * n_verts
        dof = (3 * tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)  # (T,12)
        self.dof = dof
        self.rows = np.repeat(dof, 12, axis=1)  # (T,144): row index of H^e[p, q] is dof[p]
        self.cols = np.tile(dof, (1, 12))       # (T,144): col index is dof[q]

    def gradient(self, ge, vertex_terms):
        """g = sum_e S_e^T g^e + per-vertex terms (N,3) -> (3N,)."""
        g = np.asarray(vertex_terms, dtype=np.float64).reshape(-1).copy()
        np.add.at(g, self.dof.reshape(-1), ge.reshape(-1))
        return g

    def hessian(self, He, diag, idx=None):
        """sum_{e in idx} S_e^T H^e S_e + diag(diag) as CSR (diag: (3N,) or None)."""
        if idx is None:
            rows, cols = self.rows.reshape(-1), self.cols.reshape(-1)
        else:
            rows, cols = self.rows[idx].reshape(-1), self.cols[idx].reshape(-1)
        data = He.reshape(-1)
        if diag is not None:
            d = np.arange(self.n)
            rows = np.concatenate([rows, d])
            cols = np.concatenate([cols, d])
            data = np.concatenate([data, np.asarray(diag, dtype=np.float64)])
        return sp.coo_matrix((data, (rows, cols)), shape=(self.n, self.n)).tocsr()


def diagonal_blocks(H):
    """The 3x3 diagonal blocks H_ii of a global matrix, (N,3,3)."""
    n = H.shape[0] // 3
    out = np.empty((n, 3, 3))
    base = 3 * np.arange(n)
    for r in range(3):
        for c in range(3):
            out[:, r, c] = np.asarray(H[base + r, base + c]).ravel()
    return out
