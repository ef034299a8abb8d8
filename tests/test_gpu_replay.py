"""Replay parity: the oracle's run, iteration by iteration, through the GPU.

For every Newton iteration k of an oracle run, the oracle's iterate x^k and
delta go into one GPU iteration (ppn_debug_iterate) started from the same
step state.  The GPU's projected set must equal the oracle's bit for bit, its
final indefiniteness flag must agree and the delta it carries on must be the
oracle's next delta_in (within the last bits of |g|_inf, from which both are
built by powers of two).  Each inner round is replayed through the selection
on the GPU's own gradient at x^k: with the round's delta, the number of
elements above it is the oracle's cumulative count (deltas decrease, so the
rounds' sets are nested).  This checks each iteration's decisions on their
own, apart from any drift along the trajectory.
"""
import math

import numpy as np
import pytest

import oracle
from scenes import cube_compress

from helpers import gpu_scene

pytestmark = pytest.mark.gpu


def _oracle_run(sc, mode):
    states = []
    prm = oracle.Params(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol)
    states.append((sc.x0.copy(), sc.v0.copy()))
    _, stats = oracle.run_scene(sc, mode, params=prm, trace=True, record_x=True,
                                callback=lambda n, s, st: states.append((s.x.copy(), s.v.copy())))
    return stats, states


@pytest.mark.parametrize("mode", ["PPN", "PN"])
def test_replay_every_iteration(mode):
    sc = cube_compress(n=6, n_steps=8, ramp_steps=8)
    stats, states = _oracle_run(sc, mode)
    g = gpu_scene(sc)
    alpha, eps_delta = 0.5, 1e-12
    n_iter = n_rounds = 0
    for n, st in enumerate(stats, start=1):
        x_n, v_n = states[n - 1]
        g.ppn_set_state(x_n, v_n)
        g.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(n))
        recs = [r for r in st.trace if "projected_idx" in r]
        for i, r in enumerate(recs):
            tag = (mode, n, r["k"])
            mask, delta_out, ind = g.ppn_debug_iterate(r["x"], r["delta_in"], mode)
            assert np.array_equal(np.nonzero(mask)[0], r["projected_idx"]), tag
            o_ind = r["rounds"][-1][2] if r["rounds"] else r["first"][0]
            assert ind == o_ind, tag
            if i + 1 < len(recs):
                want = recs[i + 1]["delta_in"]
                if math.isinf(want):
                    assert math.isinf(delta_out), tag
                else:
                    assert abs(delta_out - want) <= 1e-14 * want, (tag, delta_out, want)
            if r["rounds"]:
                grad = g.ppn_eval_gradient(r["x"])
                cum = 0
                for delta, n_sel, _, _ in r["rounds"]:
                    cum += n_sel
                    m, cnt = g.ppn_select(grad, delta, None)
                    assert cnt == cum or (delta <= eps_delta and cnt == sc.n_tets), (tag, delta, cnt, cum)
                    n_rounds += 1
            n_iter += 1
    g.close()
    assert n_iter > 20
    if mode == "PPN":
        assert n_rounds > 0 and sum(s.projected for s in stats) > 0
