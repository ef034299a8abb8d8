"""HIP-graph capture of each Newton iteration's evaluation (element quantities,
assembly, gradient norms): a scene stepped with the graph (captured at its
first evaluation, then replayed every Newton iteration, with the scene's own
eager work, line searches and solves between the replays) against the same
scene stepped with plain launches, bit for bit, over several time steps in all
three modes and both precisions; and the stage entry points, which evaluate
through the same graph, against plain launches."""
import numpy as np
import pytest

from paper_2505_21013_amd import PPN_FP64, PPN_MIXED, run_steps
from scenes import cube_compress

from helpers import gpu_scene, squashed_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [PPN_FP64, PPN_MIXED])
@pytest.mark.parametrize("mode", ["PN", "PDN", "PPN"])
def test_graph_replays_match_plain_launches(mode, precision):
    sc = cube_compress(n=6, n_steps=6, ramp_steps=6)
    runs = {}
    for graphs in (0, 1):
        g = gpu_scene(sc, precision=precision, use_graphs=graphs)
        st = run_steps(g, sc, mode, sc.n_steps)
        runs[graphs] = (st, g.ppn_get_state())
        g.close()
    (s0, (x0, v0)), (s1, (x1, v1)) = runs[0], runs[1]
    assert sum(s["newton_iters"] for s in s1) > sc.n_steps  # many replays
    for a, b in zip(s0, s1):
        for k in ("status", "newton_iters", "pcg_iters", "projected", "res_l2", "res_inf"):
            assert a[k] == b[k], (k, a[k], b[k])
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)


def test_graph_stage_entry_points_match_plain_launches():
    sc = cube_compress(n=5, n_steps=4, ramp_steps=4)
    x = squashed_state(sc, seed=3)
    out = {}
    for graphs in (0, 1):
        g = gpu_scene(sc, use_graphs=graphs)
        out[graphs] = [g.ppn_eval_gradient(x) for _ in range(3)] + [g.ppn_solve(x)[0]]
        g.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
