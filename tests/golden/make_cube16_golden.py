"""Writes cube16_compress_oracle.json: the FP64 oracle's per-step record of the
16^3-cell compressed cube (24,576 tets, the 64^3 workload's schedule at lower
resolution) over all 50 steps in PN, PDN and PPN.  Calls only the oracle and
the scene generator.  Run from the repository root:

    python tests/golden/make_cube16_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenes import cube_compress  # noqa: E402

SAMPLE = 200  # vertices whose final positions are stored


def main():
    sc = cube_compress(n=16, n_steps=50, ramp_steps=50)
    rng = np.random.default_rng(16)
    sample = np.sort(rng.choice(sc.n_verts, SAMPLE, replace=False))
    out = {"scene": "cube_compress(n=16, n_steps=50, ramp_steps=50)", "sample_vertices": sample.tolist(),
           "modes": {}}
    for mode in ("PPN", "PDN", "PN"):
        stp, stats = oracle.run_scene(sc, mode)
        out["modes"][mode] = {
            "steps": [dict(newton_iters=s.newton_iters, projected=s.projected, inner_rounds=s.inner_rounds,
                           indefinite_solves=s.indefinite_solves, converged=bool(s.converged),
                           res0_l2=s.res0_l2, res_l2=s.res_l2) for s in stats],
            "final_x_sample": stp.x[sample].tolist(),
        }
        print(mode, [s.newton_iters for s in stats], flush=True)
    with open(os.path.join(HERE, "cube16_compress_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
