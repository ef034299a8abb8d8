"""Block-Jacobi preconditioned conjugate gradients that reports indefiniteness
(oracle; test infrastructure only).

Sec. 4.1 (Linear Solvers): PCG monitors d^T H d for every search direction d
and stops as soon as a direction of non-positive curvature appears; every
solve starts from the zero vector.  Sec. 5.1: 3x3 block-diagonal
preconditioner, relative residual tolerance |r| / |r^0| = 1e-4.

Readings for what the paper leaves open:
* the residual norm is the unpreconditioned 2-norm; with x_0 = 0, r^0 = b;
* indefinite iff d^T H d <= 0 (exact comparison with zero);
* a 3x3 diagonal block of H that fails Sylvester's criterion proves H
  indefinite (it is a principal submatrix) and is reported before iterating;
  r^T z <= 0 after a preconditioner application is reported likewise;
* ``iters`` counts products H d; at the cap the current iterate is returned
  with ind = False.
Preconditioned CG itself is the textbook recurrence (Nocedal & Wright,
Algorithm 5.3).
"""
import numpy as np


def sylvester_ok(B):
    """Leading principal minors of each 3x3 block are all positive."""
    m1 = B[:, 0, 0]
    m2 = B[:, 0, 0] * B[:, 1, 1] - B[:, 0, 1] * B[:, 1, 0]
    m3 = np.linalg.det(B)
    return (m1 > 0) & (m2 > 0) & (m3 > 0)


def pcg_block_jacobi(H, b, diag_blocks, rtol=1e-4, maxit=10000):
    """Solve H x = b.  Returns (x, ind, iters)."""
    n = b.size
    x = np.zeros(n)
    if not np.all(sylvester_ok(diag_blocks)):
        return x, True, 0
    Pinv = np.linalg.inv(diag_blocks)

    def precond(v):
        return np.einsum("nij,nj->ni", Pinv, v.reshape(-1, 3)).reshape(-1)

    r = b.copy()
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return x, False, 0
    z = precond(r)
    rz = r @ z
    if rz <= 0.0:
        return x, True, 0
    d = z.copy()
    for j in range(maxit):
        q = H @ d
        kappa = d @ q
        if kappa <= 0.0:
            return x, True, j + 1
        alpha = rz / kappa
        x += alpha * d
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * r0:
            return x, False, j + 1
        z = precond(r)
        rz_new = r @ z
        if rz_new <= 0.0:
            return x, True, j + 1
        beta = rz_new / rz
        rz = rz_new
        d = z + beta * d
    return x, False, maxit
