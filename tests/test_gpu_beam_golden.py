"""The twisted beam (122,880 tets) over its whole 100-step schedule in PN, PDN
and PPN, against the oracle's record in tests/golden/beam_twist_<MODE>.json
(written by make_beam_golden.py from the oracle only): per step the same
status, Newton-iteration, projection and inner-round counts and the final
residual within 1e-10 of the step's initial residual; per Newton iteration the
same projected element set (fingerprint: count, sum and sum of squares of the
element ids); sampled positions after steps 25, 50, 75 and 100 within 1e-6 of
the bounding-box diagonal.  Hard steps (tests/helpers.py: the oracle needs 50
or more Newton iterations; step 95 in PPN and PDN, steps 93 to 96 in PN) are
held, with every step after them, to the same status and counts within 5%; a
checkpoint after a hard step (step 100), whose state two valid runs reach
along different Newton paths, is held to the bound of the Newton stopping
rule that the mode-independence pin of the oracle uses, 10 h tol (3.3e-4 m
here)."""
import json
import os

import numpy as np
import pytest

from paper_2505_21013_amd import run_steps
from scenes import config

from helpers import check_hard_step, first_hard_step, gpu_scene

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _fingerprint(ids):
    ids = np.asarray(ids, dtype=np.int64)
    return [int(ids.size), int(ids.sum()), int((ids * ids).sum())]


@pytest.mark.parametrize("mode", ["PPN", "PDN", "PN"])
def test_beam_schedule_matches_oracle(mode):
    path = os.path.join(HERE, "golden", f"beam_twist_{mode}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_beam_golden.py {mode})")
    with open(path) as f:
        gold = json.load(f)
    sc = config(1)
    sample = np.array(gold["sample_vertices"])
    n_steps = len(gold["steps"])
    gpu = gpu_scene(sc, trace=True)
    masks, snaps = [], {}

    def cb(n, s, st):
        masks.append([_fingerprint(r["projected_ids"]) for r in s.ppn_trace()])
        if str(n) in gold["x_sample"]:
            snaps[str(n)] = s.ppn_get_positions()[sample]
    stats = run_steps(gpu, sc, mode, n_steps, callback=cb)
    gpu.close()
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    first_hard = first_hard_step(gold["steps"])
    rel_own = []
    for n, (g, o) in enumerate(zip(stats, gold["steps"])):
        tag = (mode, n + 1)
        if n + 1 >= first_hard:
            check_hard_step(tag, g, o)
            print(f"beam {mode} step {n + 1} (from the first hard step on): newton {g['newton_iters']} (oracle {o['newton_iters']}), "
                  f"projected {g['projected']} (oracle {o['projected']})")
            continue
        assert (g["status"] == "PPN_OK") == o["converged"], (tag, g["status"])
        assert g["newton_iters"] == o["newton_iters"], (tag, g["newton_iters"], o["newton_iters"])
        assert g["projected"] == o["projected"], (tag, g["projected"], o["projected"])
        assert g["inner_rounds"] == o["inner_rounds"], tag
        assert abs(g["res_l2"] - o["res_l2"]) <= 1e-10 * o["res0_l2"], (tag, g["res_l2"], o["res_l2"])
        rel_own.append(abs(g["res_l2"] - o["res_l2"]) / o["res_l2"])
        assert masks[n] == o["masks"], tag
    rel_own = np.array(rel_own)
    print(f"beam {mode}: final residual against the oracle's, relative to the oracle's own final residual, "
          f"over steps 1..{first_hard - 1}: median {np.median(rel_own):.2e}, max {rel_own.max():.2e}")
    for k, xs in gold["x_sample"].items():
        err = float(np.max(np.abs(snaps[k] - np.array(xs))))
        bar = 1e-6 * diag if int(k) < first_hard else 10 * sc.dt * sc.stop_tol
        print(f"beam {mode} positions after step {k}: {err:.2e} m (bar {bar:.1e} m)")
        assert err <= bar, (mode, k, err)
