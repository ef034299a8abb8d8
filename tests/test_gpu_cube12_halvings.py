"""Line-search decisions of PPN against the oracle where they matter: the
compressed heterogeneous cube at 12^3 cells (10,368 tets) over its 50-step
schedule, whose last steps (42..50) make the backtracking line search (Sec.
5.1) cut nine Newton steps to 1/2 .. 1/16.  Against the oracle's record
tests/golden/cube12_halvings_PPN.json (make_halvings_record.py, oracle only):
the same Newton count on every step, and on steps 35..50 the same accepted
step size (an exact power of two) and the same number of projected elements at
every Newton iteration.  No step of this run needs 50 or more Newton
iterations (the most is 40), so every count is held exactly."""
import json
import os

import pytest

from paper_2505_21013_amd import run_steps
from scenes import cube_compress

from helpers import gpu_scene

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube12_halvings_PPN.json")


def test_cube12_line_search_decisions_match_the_oracle():
    gold = json.load(open(GOLD))
    first = gold["steps_analysed"][0]
    assert max(s["newton_iters"] for s in gold["steps"]) < 50
    sc = cube_compress(n=12, n_steps=50, ramp_steps=50)
    gpu = gpu_scene(sc, trace=True)
    traces = {}

    def cb(n, s, st):
        if n >= first:
            traces[n] = s.ppn_trace()
    stats = run_steps(gpu, sc, "PPN", len(gold["steps"]), callback=cb)
    gpu.close()
    halvings = 0
    for n, (g, o) in enumerate(zip(stats, gold["steps"]), start=1):
        assert g["newton_iters"] == o["newton_iters"], (n, g["newton_iters"], o["newton_iters"])
        assert (g["status"] == "PPN_OK") == o["converged"], (n, g["status"])
        if n < first:
            continue
        # the record holds the iterations with a line search (all but a converged last one)
        tr = [r for r in traces[n] if r["k"] in {i["k"] for i in o["iters"]}]
        assert [r["k"] for r in tr] == [i["k"] for i in o["iters"]], n
        for r, i in zip(tr, o["iters"]):
            assert r["gamma"] == i["gamma"], (n, i["k"], r["gamma"], i["gamma"])
            assert r["n_projected"] == i["n_projected"], (n, i["k"], r["n_projected"], i["n_projected"])
            halvings += i["gamma"] < 1.0
    print(f"cube12: {halvings} halved Newton steps on steps {first}..50, all matched")
    assert halvings == sum(i["gamma"] < 1.0 for s in gold["steps"] for i in s["iters"]) > 0
