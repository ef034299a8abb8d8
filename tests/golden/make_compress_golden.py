"""Writes cube<n>_compress_<MODE>.json: the FP64 oracle's record of the
compressed heterogeneous cube (n^3 cells, E log-uniform per element in
[1e4, 1e6] Pa, nu 0.48, top face pushed down 60% over 50 steps) over its first
``steps`` time steps in one mode.  Per step: status, Newton, projection,
inner-round and indefinite-solve counts, initial and final residual; per Newton
iteration: |g|_2, |g|_inf, |dx|_inf, the accepted step size and a fingerprint
of the projected element set (count, sum of ids, sum of squared ids); sampled
positions after every step.  Calls only the oracle and the scene generator.
The record is rewritten after every step, so a long run leaves a usable prefix.
Run from the repository root, one process per (n, mode):

    python tests/golden/make_compress_golden.py 64 PPN 2 ids  # the 1,572,864-tet cube, steps 1-2
    python tests/golden/make_compress_golden.py 32 PPN 46     # 196,608 tets, through the breakdown

With "ids", every Newton iteration also stores its projected element ids
(ascending), so that a run can count the elements on which its projected set
differs from the oracle's.

With "renumber SEED", the oracle steps the same scene numbered at random
(scenes.renumbered) and writes cube<n>_compress_<MODE>_renum<SEED>.json with its
per-step counts only: the same mathematics summed in other orders, which shows
from which step on the scene's Newton path is decided by rounding.

    python tests/golden/make_compress_golden.py 32 PPN 46 renumber 1
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenes import cube_compress, renumbered  # noqa: E402

SAMPLE = 200  # vertices whose positions are stored after every step


def fingerprint(ids):
    ids = np.asarray(ids, dtype=np.int64)
    return [int(ids.size), int(ids.sum()), int((ids * ids).sum())]


def main(n, mode, steps, with_ids=False):
    sc = cube_compress(n=n, n_steps=50, ramp_steps=50)
    rng = np.random.default_rng(n)
    sample = np.sort(rng.choice(sc.n_verts, SAMPLE, replace=False))
    path = os.path.join(HERE, f"cube{n}_compress_{mode}.json")
    out = {"scene": f"cube_compress(n={n}, n_steps=50, ramp_steps=50)", "mode": mode,
           "sample_vertices": sample.tolist(), "steps": []}
    t_last = [time.perf_counter()]

    def cb(k, s, st):
        now = time.perf_counter()
        out["steps"].append(dict(
            newton_iters=st.newton_iters, projected=st.projected, inner_rounds=st.inner_rounds,
            indefinite_solves=st.indefinite_solves, solves=st.solves, pcg_iters=st.pcg_iters,
            converged=bool(st.converged), ls_fail=bool(st.ls_fail), res0_l2=st.res0_l2,
            res_l2=st.res_l2, res_inf=st.res_inf, oracle_seconds=now - t_last[0],
            iters=[dict(g_l2=r["g_l2"], g_inf=r["g_inf"], dx_inf=r.get("dx_inf"), gamma=r.get("gamma"),
                        rounds=len(r["rounds"]),
                        mask=fingerprint(r.get("projected_idx", np.zeros(0, np.int64))),
                        **({"ids": r.get("projected_idx", np.zeros(0, np.int64)).tolist()} if with_ids else {}))
                   for r in st.trace],
            x_sample=s.x[sample].tolist()))
        t_last[0] = now
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(out, f)
        os.replace(tmp, path)
        print(mode, k, st.newton_iters, st.projected, st.pcg_iters, bool(st.converged),
              f"{out['steps'][-1]['oracle_seconds']:.1f}s", flush=True)

    oracle.run_scene(sc, mode, n_steps=steps, trace=True, callback=cb)


def main_renumbered(n, mode, steps, seed):
    sc = renumbered(cube_compress(n=n, n_steps=50, ramp_steps=50), seed)
    path = os.path.join(HERE, f"cube{n}_compress_{mode}_renum{seed}.json")
    out = {"scene": f"renumbered(cube_compress(n={n}, n_steps=50, ramp_steps=50), {seed})", "mode": mode,
           "steps": []}

    def cb(k, s, st):
        out["steps"].append(dict(newton_iters=st.newton_iters, projected=st.projected,
                                 inner_rounds=st.inner_rounds, converged=bool(st.converged)))
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(out, f)
        os.replace(tmp, path)
        print(mode, "renumbered", seed, k, st.newton_iters, st.projected, bool(st.converged), flush=True)

    oracle.run_scene(sc, mode, n_steps=steps, callback=cb)


if __name__ == "__main__":
    if len(sys.argv) > 5 and sys.argv[4] == "renumber":
        main_renumbered(int(sys.argv[1]), sys.argv[2], int(sys.argv[3]), int(sys.argv[5]))
    else:
        main(int(sys.argv[1]), sys.argv[2], int(sys.argv[3]), len(sys.argv) > 4 and sys.argv[4] == "ids")
