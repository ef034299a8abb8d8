"""Timed sample of the oracle for the benchmark's CPU baseline (test infrastructure only).

The oracle is far too slow to run whole time steps of the 1.57M-tet workload
inside a benchmark, so it is timed on a bounded sample of that workload and the
per-unit costs are scaled up:

* element evaluation (psi, g^e, H^e) and COO->CSR assembly of `n_sample`
  consecutive elements of the mesh at the step-1 state, per element;
* eigenvalue clamping of `n_proj` of those element Hessians, per element;
* 10 PCG iterations on the assembled partial operator, per stored nonzero;
* one line-search energy difference over the sampled elements, per element.

`per_step_seconds(costs, counts)` combines them with the per-step operation
counts of a run (Newton iterations, PCG iterations, projections, line-search
trials), which the algorithm fixes independently of the hardware.

Run as ``python -m oracle.baseline --config 2`` (prints JSON).
"""
import argparse
import json
import os
import time

import numpy as np

from .assemble import diagonal_blocks
from .fem import element_grad_hess, element_psi
from .newton import Params, Stepper
from .pcg import pcg_block_jacobi
from .project import project_to_pd


def sample_costs(sc, n_sample=1572864, n_proj=300000, pcg_iters=100):
    stp = Stepper(sc.X, sc.tets, sc.E, sc.nu, sc.rho, sc.dt, sc.gravity, sc.dirichlet_ids,
                  Params(), x0=sc.x0, v0=sc.v0)
    stp.set_targets(sc.targets(1))
    stp.xhat = stp.x + sc.dt * stp.v + sc.dt ** 2 * np.asarray(sc.gravity)[None]
    T = sc.n_tets
    n_sample = min(n_sample, T)
    idx = np.arange(n_sample)
    x = stp.x

    t = time.perf_counter()
    ge, He = element_grad_hess(stp.mesh, x, idx)
    H = stp.asm.hessian(He, stp._diag(), idx=idx)
    t_eval = (time.perf_counter() - t) / n_sample

    npj = min(n_proj, n_sample)
    t = time.perf_counter()
    project_to_pd(He[:npj], 1e-8)
    t_proj = (time.perf_counter() - t) / npj

    g = np.ones(H.shape[0])
    t = time.perf_counter()
    pcg_block_jacobi(H, -g, diagonal_blocks(H), rtol=1e-300, maxit=pcg_iters)
    t_pcg_nnz = (time.perf_counter() - t) / pcg_iters / H.nnz

    sub = type(stp.mesh)(X=stp.mesh.X, tets=stp.mesh.tets[idx], Bm=stp.mesh.Bm[idx], V=stp.mesh.V[idx],
                         mu=stp.mesh.mu[idx], lam=stp.mesh.lam[idx])
    dx = np.full_like(x, 1e-4)
    t = time.perf_counter()
    element_psi(sub, x + dx).sum() - element_psi(sub, x).sum()
    t_ls = (time.perf_counter() - t) / n_sample

    pairs = np.concatenate([np.sort(sc.tets[:, [a, c]], axis=1).astype(np.int64)
                            for a in range(4) for c in range(a + 1, 4)])
    n_edges = np.unique(pairs[:, 0] * sc.n_verts + pairs[:, 1]).size
    nnz_full = 9 * (2 * n_edges + sc.n_verts)
    return dict(t_eval_per_elem=t_eval, t_proj_per_elem=t_proj, t_pcg_per_nnz=t_pcg_nnz,
                t_ls_per_elem=t_ls, n_tets=T, nnz_full=nnz_full, n_sample=n_sample, n_proj=npj,
                pcg_iters_timed=pcg_iters, threads=int(os.environ.get("OMP_NUM_THREADS", "1")))


def per_step_seconds(c, counts):
    """Oracle seconds for one time step with the given per-step counts."""
    T = c["n_tets"]
    return (counts["newton_iters"] * c["t_eval_per_elem"] * T
            + counts["pcg_iters"] * c["t_pcg_per_nnz"] * c["nnz_full"]
            + counts["projected"] * c["t_proj_per_elem"]
            + counts["ls_trials"] * c["t_ls_per_elem"] * T)


def cpu_model():
    """The host CPU's model name (Linux), else the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--n-sample", type=int, default=1572864)
    ap.add_argument("--cpu", type=int, default=None, help="pin the process to this core")
    a = ap.parse_args()
    if a.cpu is not None:
        os.sched_setaffinity(0, {a.cpu})
    from scenes import config
    t = time.perf_counter()
    c = sample_costs(config(a.config), n_sample=a.n_sample)
    c["wall_s"] = time.perf_counter() - t
    c["cpu_model"] = cpu_model()
    c["pinned_core"] = a.cpu
    c["cores_allowed"] = sorted(os.sched_getaffinity(0))
    c["host_cpus"] = os.cpu_count()
    print(json.dumps(c))


if __name__ == "__main__":
    main()
