"""Determinism, checkpoint / restore, rejected inputs and forced failure paths.

* Two fresh scenes stepping the same schedule produce identical bits.
* A run restored from a checkpoint (positions and velocities after step 3)
  continues with the same bits as the uninterrupted run.
* Non-finite states and targets, inverted rest tetrahedra, vertices outside
  every tetrahedron, repeated or out-of-range vertex indices and out-of-range
  parameters are rejected with the documented status before anything runs.
* Forced fallback to PN (alpha so small that delta drops below eps_delta within
  the first inner rounds) and forced line-search failure (Armijo constant
  near 1, few halvings) take the same path as the oracle, which runs with the
  same parameters.
"""
import numpy as np
import pytest

import oracle
from paper_2505_21013_amd import PPNError, Scene, run_steps
from scenes import cube_compress, kuhn_grid

from helpers import gpu_scene
from test_gpu_e2e import _compare

pytestmark = pytest.mark.gpu


def _scene():
    return cube_compress(n=6, n_steps=8, ramp_steps=8)


def test_two_runs_identical_bits():
    sc = _scene()
    out = []
    for _ in range(2):
        g = gpu_scene(sc)
        st = run_steps(g, sc, "PPN", 5)
        out.append((g.ppn_get_state(), [(s["newton_iters"], s["pcg_iters"], s["projected"], s["res_l2"]) for s in st]))
        g.close()
    (x0, v0), s0 = out[0]
    (x1, v1), s1 = out[1]
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1) and s0 == s1


def test_checkpoint_restore_continues_with_same_bits():
    sc = _scene()
    g = gpu_scene(sc)
    run_steps(g, sc, "PPN", 3)
    ck = g.ppn_get_state()
    run_steps(g, sc, "PPN", 3, first_step=4)
    want = g.ppn_get_state()
    g.close()
    h = gpu_scene(sc)
    h.ppn_set_state(*ck)
    run_steps(h, sc, "PPN", 3, first_step=4)
    got = h.ppn_get_state()
    h.close()
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])


def _code(fn):
    with pytest.raises(PPNError) as e:
        fn()
    return e.value.code


def test_bad_inputs_are_rejected():
    sc = _scene()
    g = gpu_scene(sc)
    x, v = g.ppn_get_state()
    bad = x.copy()
    bad[3, 1] = np.nan
    assert _code(lambda: g.ppn_set_state(bad, v)) == -5  # PPN_ERR_STATE
    t = sc.targets(1).copy()
    t[0, 0] = np.inf
    assert _code(lambda: g.ppn_set_dirichlet(sc.dirichlet_ids, t)) == -1
    ids = sc.dirichlet_ids.copy()
    ids[1] = ids[0]
    assert _code(lambda: g.ppn_set_dirichlet(ids, sc.targets(1))) == -1  # repeated id
    assert _code(lambda: g.ppn_set_params(alpha=1.5)) == -1
    assert _code(lambda: g.ppn_set_params(eig_mirror=2)) == -1
    assert _code(lambda: g.ppn_set_material(1000.0, 1e5, 0.5)) == -1  # nu must be < 0.5
    # the state is untouched by the rejected calls
    x2, v2 = g.ppn_get_state()
    assert np.array_equal(x, x2) and np.array_equal(v, v2)
    g.close()
    # an inverted rest tetrahedron
    X, tets = kuhn_grid(2, 2, 2)
    tets = tets.copy()
    tets[5, [1, 2]] = tets[5, [2, 1]]
    s = Scene()
    assert _code(lambda: (s.ppn_load_mesh(X, tets), s.ppn_set_material(1000.0, 1e5, 0.45))) == -2
    s.close()
    # a vertex that belongs to no tetrahedron (singular diagonal block)
    X2 = np.vstack([X, X[-1:] + 1.0])
    s = Scene()
    with pytest.raises(PPNError, match="belongs to no tetrahedron") as e:
        s.ppn_load_mesh(X2, kuhn_grid(2, 2, 2)[1])
    assert e.value.code == -2
    s.close()
    # a tet that repeats a vertex; an index out of range
    bad = kuhn_grid(2, 2, 2)[1].copy()
    bad[0, 1] = bad[0, 0]
    s = Scene()
    assert _code(lambda: s.ppn_load_mesh(X, bad)) == -2
    bad = kuhn_grid(2, 2, 2)[1].copy()
    bad[3, 2] = len(X)
    assert _code(lambda: s.ppn_load_mesh(X, bad)) == -2
    s.close()


def test_forced_pn_fallback_matches_oracle():
    # alpha = 1e-3: delta shrinks by 1e3 per inner round and reaches eps_delta
    # within a few rounds, after which every remaining element is projected
    _compare(_scene(), "PPN", 8, alpha=1e-3)


def test_forced_line_search_failure_matches_oracle():
    sc = _scene()
    prm = dict(armijo_c=0.999999, ls_maxit=3)
    ox = []
    _, ost = oracle.run_scene(sc, "PPN", n_steps=1, params=oracle.Params(
        stop_mode=sc.stop_mode, stop_tol=sc.stop_tol, **prm),
        callback=lambda n, s, o: ox.append(s.x.copy()))
    g = gpu_scene(sc, **prm)
    st = run_steps(g, sc, "PPN", 1)[0]
    x = g.ppn_get_positions()
    g.close()
    o = ost[0]
    assert o.ls_fail and st["status"] == "PPN_WARN_LS_FAIL" and st["ls_fail"] == 1
    assert st["newton_iters"] == o.newton_iters and st["ls_backtracks"] == o.ls_backtracks
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    assert float(np.max(np.abs(x - ox[0]))) <= 1e-6 * diag
