"""Writes batch_scenes_PPN.json: the FP64 oracle's record of every scene of the
64-scene batch workload (rotated cubes and beams, seed 3) with at most 30,000
tets, over its 20-step schedule in PPN: per step the status, Newton and
projection counts and the initial and final residuals, and sampled positions
after the last step.

Each scene is also run by the oracle numbered at random (scenes.renumbered,
seeds 1 and 2): the same mathematics with other summation orders.  Their
per-step Newton counts are kept, and the first step at which one of them
differs from the record ("sensitive_from") marks where the scene's Newton
path is decided by rounding: two correct implementations need not agree on
counts from that step on.

Calls only the oracle and the scene generator.  Run from the repository root
(about 20 minutes on eight cores):

    python tests/golden/make_batch_golden.py
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenes import batch_scenes, renumbered  # noqa: E402

MAX_TETS = 30000
SAMPLE = 100
RENUMBER_SEEDS = (1, 2)


def one(k):
    sc = batch_scenes()[k]
    rng = np.random.default_rng(1000 + k)
    sample = np.sort(rng.choice(sc.n_verts, min(SAMPLE, sc.n_verts), replace=False))
    stp, stats = oracle.run_scene(sc, "PPN")
    counts = [s.newton_iters for s in stats]
    renum = {}
    for seed in RENUMBER_SEEDS:
        _, st = oracle.run_scene(renumbered(sc, seed), "PPN")
        renum[str(seed)] = [s.newton_iters for s in st]
    differ = [n + 1 for n in range(len(counts)) if any(r[n] != counts[n] for r in renum.values())]
    rec = {"index": k, "n_tets": int(sc.n_tets), "sample_vertices": sample.tolist(),
           "steps": [dict(newton_iters=s.newton_iters, projected=s.projected, converged=bool(s.converged),
                          res0_l2=s.res0_l2, res_l2=s.res_l2) for s in stats],
           "final_x_sample": stp.x[sample].tolist(),
           "newton_iters_renumbered": renum,
           "sensitive_from": differ[0] if differ else None}
    print(sc.name, sc.n_tets, counts, renum, flush=True)
    return sc.name, rec


def main():
    ks = [k for k, sc in enumerate(batch_scenes()) if sc.n_tets <= MAX_TETS]
    out = {"scenes": "batch_scenes() with at most 30000 tets", "mode": "PPN",
           "renumber_seeds": list(RENUMBER_SEEDS), "records": {}}
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        for name, rec in pool.imap(one, ks):
            out["records"][name] = rec
    tmp = os.path.join(HERE, "batch_scenes_PPN.json.tmp")
    with open(tmp, "w") as f:
        json.dump(out, f)
    os.replace(tmp, os.path.join(HERE, "batch_scenes_PPN.json"))


if __name__ == "__main__":
    main()
