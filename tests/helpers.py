"""Shared set-up for parity tests: the same seeded scene loaded into the oracle and the GPU."""
import numpy as np

from oracle.fem import predictor
from oracle.newton import Params, Stepper


def oracle_stepper(sc, step=1, **params):
    p = Params(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol, **params)
    s = Stepper(sc.X, sc.tets, sc.E, sc.nu, sc.rho, sc.dt, sc.gravity, sc.dirichlet_ids, p,
                x0=sc.x0, v0=sc.v0)
    s.set_targets(sc.targets(step))
    s.xhat = predictor(s.x, s.v, s.h, s.gravity)
    return s


def gpu_scene(sc, step=1, trace=False, precision=0, **params):
    from paper_2505_21013_amd import scene_from
    s = scene_from(sc, params=params or None, trace=trace, precision=precision)
    s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(step))
    return s


def squashed_state(sc, squash=0.55, noise=0.08, seed=0):
    """A deformed configuration with inverted / indefinite elements: z scaled
    towards the bottom plus seeded noise of `noise` cells."""
    rng = np.random.default_rng(seed)
    cell = float(np.min(np.array(sc.meta["size"]) / np.array(sc.meta["cells"])))
    x = sc.X.copy()
    x[:, 2] *= squash
    x += noise * cell * rng.uniform(-1, 1, size=x.shape)
    return x


def bsr_to_dense(rp, col, vals, n):
    H = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = col[k]
            H[3 * i:3 * i + 3, 3 * j:3 * j + 3] = vals[k]
    return H


def bsr_to_csr(rp, col, vals, n):
    import scipy.sparse as sp
    return sp.bsr_matrix((vals, col, rp), shape=(3 * n, 3 * n)).tocsr()
