"""Writes beam_twist_<MODE>.json: the FP64 oracle's record of the twisted beam
(80x16x16 cells, 122,880 tets, 2 turns over 100 steps) over all 100 steps in one
mode: per-step counts and residuals, a fingerprint of the projected element set
of every Newton iteration (count, sum of ids, sum of squared ids), and sampled
positions after steps 25, 50, 75 and 100.  Calls only the oracle and the scene
generator.  Run from the repository root, one process per mode:

    python tests/golden/make_beam_golden.py PPN
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenes import config  # noqa: E402

SAMPLE = 200
CHECKPOINTS = (25, 50, 75, 100)


def fingerprint(ids):
    ids = np.asarray(ids, dtype=np.int64)
    return [int(ids.size), int(ids.sum()), int((ids * ids).sum())]


def main(mode):
    sc = config(1)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(sc.n_verts, SAMPLE, replace=False))
    snaps = {}

    def cb(n, s, st):
        if n in CHECKPOINTS:
            snaps[str(n)] = s.x[sample].tolist()
        print(mode, n, st.newton_iters, st.projected, flush=True)

    _, stats = oracle.run_scene(sc, mode, trace=True, callback=cb)
    out = {"scene": "config(1)", "mode": mode, "sample_vertices": sample.tolist(), "x_sample": snaps,
           "steps": [dict(newton_iters=s.newton_iters, projected=s.projected, inner_rounds=s.inner_rounds,
                          indefinite_solves=s.indefinite_solves, converged=bool(s.converged),
                          res0_l2=s.res0_l2, res_l2=s.res_l2,
                          masks=[fingerprint(r.get("projected_idx", np.zeros(0, np.int64))) for r in s.trace])
                     for s in stats]}
    with open(os.path.join(HERE, f"beam_twist_{mode}.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main(sys.argv[1])
