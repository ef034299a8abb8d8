"""Projection of an element Hessian to the SPD cone by eigenvalue clamping
(oracle; test infrastructure only).

Sec. 3, Eq. (4): H^e = Q D Q^T; the clamped matrix is Q Dhat Q^T with
Dhat_ii = max(D_ii, eps), eps > 0 (eps = 1e-8, Sec. 5.1).  The symmetric
eigendecomposition is LAPACK's (numpy.linalg.eigh), used as a library step.

Eigenvalue mirroring (the alternative filter the paper compares against in
Sec. 2 and Sec. 5): negative eigenvalues are replaced by their absolute values.
Reading: Dhat_ii = max(|D_ii|, eps), so that zero eigenvalues (the rigid
translations of an element) are still lifted to eps as with clamping.
"""
import numpy as np


def project_to_pd(H, eps=1e-8, mirror=False):
    """Clamp (or mirror, then clamp) the eigenvalues of each symmetric matrix in
    ``H`` (..., n, n) to at least ``eps``."""
    H = np.asarray(H, dtype=np.float64)
    D, Q = np.linalg.eigh(H)
    Dhat = np.maximum(np.abs(D) if mirror else D, eps)
    return np.matmul(Q * Dhat[..., None, :], np.swapaxes(Q, -1, -2))
