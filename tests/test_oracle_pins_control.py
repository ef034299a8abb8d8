"""Pins of the oracle's control logic: the projection selection of Algorithm 1,
the PDN countdown and the Armijo line search.

Each is checked against values fixed by the paper's definitions and by
closed-form mathematics, written out in this file, never against another run
of the same oracle function:

* selection (Sec. 4, projection heuristic): |S^e g|_inf over hand-chosen
  assembled gradients on a 4-tet strip, with the expected values and masks
  typed in by hand; through a whole PPN time step, the selected sets against
  the assembled gradient obtained by finite differences of the total
  potential;
* PDN (Sec. 2.2 and Sec. 5.1, countdown of 4): after the iteration that
  detects indefiniteness, exactly the next `countdown` iterations project
  every element before their first solve;
* line search (Sec. 5.1, backtracking for sufficient descent): on a quadratic
  potential the accepted step is the first 2^-m below the closed-form Armijo
  bound 2 (1 - c) (-g.dx) / (dx^T A dx).

Each test also applies plausible slips (written here, on the CPU) and shows
that they fail the same expectations.
"""
import math

import numpy as np
import pytest

from oracle.fem import element_psi
from oracle.newton import Params, Stepper, run_scene
from scenes import cube_compress


# ---------------------------------------------------------------- selection: hand-written values
# Vertices on the moment curve (t, t^2, t^3): any four with increasing t form a
# positively oriented tetrahedron (the orientation determinant is the
# Vandermonde product of the t differences).
def _strip():
    t = np.arange(7, dtype=np.float64)
    X = np.stack([t, t * t, t * t * t], axis=1) * 0.1
    # e0..e3 = consecutive quadruples; e2 and e3 reordered by 3-cycles (even
    # permutations keep the orientation) so that the vertex carrying each
    # element's largest entry sits at local slot 0, 3, 1, 2 respectively.
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4], [2, 5, 3, 4], [3, 5, 6, 4]], dtype=np.int32)
    return X, tets


# Assembled gradient, one row per vertex.  |g_v|_inf = 5, 1, 2, 3, 6, 8, 9;
# vertex 3 has the largest 2-norm of element 0 (5.196 > 5) but not its largest
# max-norm entry.
G = np.array([[5.0, 0.0, 0.0],
              [1.0, -1.0, 0.5],
              [0.0, -2.0, 0.0],
              [3.0, -3.0, 3.0],
              [0.0, 6.0, 0.0],
              [-8.0, 0.0, 1.0],
              [0.0, 0.0, -9.0]])
# |S^e g|_inf by hand: e0 = max(5, 1, 2, 3), e1 = max(1, 2, 3, 6),
# e2 = max(2, 8, 3, 6), e3 = max(3, 8, 9, 6).
S_EXPECTED = np.array([5.0, 6.0, 8.0, 9.0])
# (delta, already projected, expected newly selected) -- strict '>' at the ties
# delta = 5 and delta = 8; the eps_delta fallback selects every element not yet
# projected.
MASK_CASES = [
    (4.99, [0, 0, 0, 0], [1, 1, 1, 1]),
    (5.0, [0, 0, 0, 0], [0, 1, 1, 1]),
    (5.1, [0, 0, 0, 0], [0, 1, 1, 1]),
    (6.0, [0, 0, 0, 0], [0, 0, 1, 1]),
    (8.0, [0, 0, 0, 0], [0, 0, 0, 1]),
    (9.0, [0, 0, 0, 0], [0, 0, 0, 0]),
    (5.5, [0, 1, 0, 1], [0, 0, 1, 0]),
    (1e-12, [0, 0, 1, 0], [1, 1, 0, 1]),   # delta == eps_delta: fallback
    (1e-13, [1, 0, 0, 0], [0, 1, 1, 1]),   # below eps_delta: fallback
    (20.0, [0, 0, 0, 0], [0, 0, 0, 0]),
]


def _strip_stepper():
    X, tets = _strip()
    return Stepper(X, tets, 1e5, 0.45, 1000.0, 1 / 30, (0, 0, -9.81), np.zeros(0, np.int32),
                   Params())


def test_selection_residual_hand_values():
    s = _strip_stepper()
    assert np.array_equal(s.selection_residual(G.reshape(-1)), S_EXPECTED)


@pytest.mark.parametrize("delta,proj,expected", MASK_CASES)
def test_selection_mask_hand_values(delta, proj, expected):
    s = _strip_stepper()
    got = s.select(G.reshape(-1), delta, np.array(proj, dtype=bool))
    assert got.tolist() == [bool(v) for v in expected]


# Plausible slips in |S^e g|_inf, each shown to disagree with the hand values.
def _slip_two_norm(g, tets):
    return np.linalg.norm(g.reshape(-1, 3), axis=1)[tets].max(axis=1)


def _slip_drop_corner(k):
    def f(g, tets):
        keep = [a for a in range(4) if a != k]
        return np.abs(g.reshape(-1, 3)).max(axis=1)[tets[:, keep]].max(axis=1)
    return f


def _slip_sum_over_corners(g, tets):
    return np.abs(g.reshape(-1, 3)).max(axis=1)[tets].sum(axis=1)


def _slip_first_component(g, tets):
    return np.abs(g.reshape(-1, 3)[:, 0])[tets].max(axis=1)


@pytest.mark.parametrize("slip", [_slip_two_norm, _slip_drop_corner(0), _slip_drop_corner(1),
                                  _slip_drop_corner(2), _slip_drop_corner(3), _slip_sum_over_corners,
                                  _slip_first_component])
def test_selection_slips_fail_the_hand_values(slip):
    _, tets = _strip()
    s = slip(G.reshape(-1), tets)
    masks_ok = all(((s > d) & ~np.array(p, bool)).tolist() == [bool(v) for v in e]
                   for d, p, e in MASK_CASES if d > 1e-12)
    assert not (np.array_equal(s, S_EXPECTED) and masks_ok)


def test_selection_uses_the_assembled_gradient_not_element_gradients():
    """The residual is taken on the assembled g (R10), whose entries at a
    vertex sum the element gradients of every element around it: it differs
    from the element-local max |g^e|_inf."""
    s = _strip_stepper()
    rng = np.random.default_rng(5)
    x = s.mesh.X + 0.02 * rng.standard_normal(s.mesh.X.shape)
    from oracle.fem import element_grad
    ge = element_grad(s.mesh, x).reshape(-1, 4, 3)
    local = np.abs(ge).max(axis=(1, 2))
    s.xhat = x.copy()   # inertia term vanishes: g is the elastic sum alone
    g = s.gradient(x)
    assert not np.allclose(s.selection_residual(g), local)


# ---------------------------------------------------------------- selection through a whole PPN step
def _total_potential(s, x):
    inert = 0.5 * np.sum(s.m[:, None] / s.h ** 2 * (x - s.xhat) ** 2)
    pen = 0.5 * s.p.k_dirichlet * np.sum((x[s.dir_ids] - s.xbar) ** 2)
    return inert + element_psi(s.mesh, x).sum() + pen


def _fd_gradient(s, x, h=1e-7):
    g = np.zeros(x.size)
    for p in range(x.size):
        e = np.zeros(x.size)
        e[p] = h
        g[p] = (_total_potential(s, x + e.reshape(-1, 3)) - _total_potential(s, x - e.reshape(-1, 3))) / (2 * h)
    return g


def test_ppn_selected_sets_follow_the_assembled_gradient():
    """Through Algorithm 1 itself: at every Newton iteration that ran inner
    rounds, the projected set is {e : |S^e g|_inf > delta_last} for the
    iteration's gradient g (nested masks, Sec. 4), and the first delta of the
    step is alpha |g|_inf.  g is obtained by central differences of the total
    potential, independent of the oracle's assembly; elements within 1e-5
    (relative) of delta are not judged."""
    sc = cube_compress(n=4, n_steps=2, ramp_steps=2)
    stp, st = run_scene(sc, "PPN", n_steps=1, trace=True, record_x=True)
    s = Stepper(sc.X, sc.tets, sc.E, sc.nu, sc.rho, sc.dt, sc.gravity, sc.dirichlet_ids,
                Params(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol), x0=sc.x0, v0=sc.v0)
    s.set_targets(sc.targets(1))
    s.xhat = sc.x0 + sc.dt * sc.v0 + sc.dt ** 2 * np.asarray(sc.gravity)[None]
    tets = sc.tets
    checked = 0
    first_delta_seen = False
    for rec in st[0].trace:
        if not rec["rounds"]:
            continue
        g = _fd_gradient(s, rec["x"])
        gi = np.abs(g.reshape(-1, 3)).max(axis=1)
        sres = np.array([max(gi[v] for v in tet) for tet in tets])
        if not first_delta_seen:
            assert math.isinf(rec["delta_in"])
            assert abs(rec["rounds"][0][0] - 0.5 * np.abs(g).max()) <= 1e-6 * np.abs(g).max()
            first_delta_seen = True
        delta_last = rec["rounds"][-1][0]
        proj = np.zeros(sc.n_tets, bool)
        proj[rec["projected_idx"]] = True
        clear_above = sres > delta_last * (1 + 1e-5)
        clear_below = sres < delta_last * (1 - 1e-5)
        assert proj[clear_above].all()
        assert not proj[clear_below].any()
        # each round's new elements are those between its delta and the previous one
        total = 0
        for (delta, n_new, ind, it) in rec["rounds"]:
            total += n_new
            near = np.abs(sres - delta) <= 1e-5 * delta
            lo = np.count_nonzero(sres > delta * (1 + 1e-5))
            assert lo <= total <= lo + np.count_nonzero(near)
        checked += 1
    assert checked >= 1 and first_delta_seen


# ---------------------------------------------------------------- PDN countdown
def _pdn_trace(countdown, step):
    sc = cube_compress(n=4, n_steps=3, ramp_steps=2)
    _, st = run_scene(sc, "PDN", n_steps=step, trace=True,
                      params=Params(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol, pdn_countdown=countdown))
    return sc.n_tets, st[step - 1]


@pytest.mark.parametrize("countdown,step", [(4, 1), (4, 2), (1, 2), (8, 2)])
def test_pdn_countdown_projects_the_next_iterations(countdown, step):
    """R17: on detection at iteration k every element is projected and the
    system solved again; iterations k+1 .. k+countdown project every element
    before their first solve; iteration k+countdown+1 starts unprojected."""
    T, st = _pdn_trace(countdown, step)
    tr = st.trace
    dets = [r["k"] for r in tr if r["first"][0] and r["pre_projected"] == 0]
    assert dets, "the scene must detect indefiniteness"
    k = dets[0]
    assert tr[k]["pre_projected"] == 0 and tr[k]["n_projected"] == T
    for j in range(1, countdown + 1):
        assert tr[k + j]["pre_projected"] == T, (k, j)
        assert not tr[k + j]["first"][0]
    assert len(tr) > k + countdown + 1, "the step must run past the countdown"
    assert tr[k + countdown + 1]["pre_projected"] == 0
    for r in tr[:k]:
        assert r["pre_projected"] == 0 and r["n_projected"] == 0
    # every iteration solves (the velocity stop is tested after the solve), plus
    # one extra solve per detection; every projected iteration projects all
    assert st.solves == st.newton_iters + len(dets)
    assert st.projected == T * sum(1 for r in tr if r["n_projected"] == T)


def test_pdn_countdown_slips_fail():
    """Shifting the countdown by one either way moves the first unprojected
    iteration: the expectations above single out the stated countdown."""
    T, st = _pdn_trace(4, 1)
    tr = st.trace
    k = [r["k"] for r in tr if r["first"][0] and r["pre_projected"] == 0][0]
    pre = [r["pre_projected"] == T for r in tr]
    for wrong in (3, 5):
        expect = [k < i <= k + wrong for i in range(len(tr))]
        assert expect != pre


# ---------------------------------------------------------------- Armijo line search
def _quadratic_stepper(c=1e-4, ls_maxit=30):
    """E = 0: Psi is the inertia plus penalty terms, a quadratic with the
    diagonal Hessian A = m_i / h^2 (+ k_D on constrained vertices)."""
    sc = cube_compress(n=2, n_steps=2, ramp_steps=2)
    p = Params(armijo_c=c, ls_maxit=ls_maxit)
    s = Stepper(sc.X, sc.tets, 0.0, 0.3, 1000.0, sc.dt, sc.gravity, sc.dirichlet_ids, p,
                x0=sc.X, v0=np.zeros_like(sc.X))
    s.set_targets(sc.targets(1))
    s.xhat = sc.X + sc.dt ** 2 * np.asarray(sc.gravity)[None]
    a = np.repeat(s.m / s.h ** 2, 3).reshape(-1, 3)
    a[s.dir_ids] += s.p.k_dirichlet
    return s, a


def _armijo_expected(g, dx, a, c, ls_maxit):
    """First gamma = 2^-m (m <= ls_maxit) with gamma <= 2 (1 - c) (-g.dx) / (dx^T A dx)."""
    bound = 2.0 * (1.0 - c) * (-(g * dx).sum()) / (a * dx * dx).sum()
    for m in range(ls_maxit + 1):
        if 2.0 ** -m <= bound:
            return 2.0 ** -m, True, m
    return None, False, ls_maxit + 1


@pytest.mark.parametrize("c,scale", [(1e-4, 0.5), (1e-4, 1.0), (1e-4, 3.0), (1e-4, 5.3), (1e-4, 37.0),
                                     (1e-4, 1000.0), (0.5, 3.0), (0.3, 1.5), (0.9, 0.15), (0.6, 10.0)])
def test_armijo_accepts_the_closed_form_step_on_a_quadratic(c, scale):
    s, a = _quadratic_stepper(c=c)
    rng = np.random.default_rng(int(scale * 10))
    x = s.x + 0.01 * rng.standard_normal(s.x.shape)
    g = a * (x - s.xhat)
    g[s.dir_ids] = (s.m[s.dir_ids, None] / s.h ** 2) * (x[s.dir_ids] - s.xhat[s.dir_ids]) \
        + s.p.k_dirichlet * (x[s.dir_ids] - s.xbar)
    newton = -g / a
    dx = scale * newton   # an over-long (scale > 2) or short Newton direction
    gamma, ok, rejected = s.line_search(x, dx, g.reshape(-1))
    eg, eok, em = _armijo_expected(g, dx, a, s.p.armijo_c, s.p.ls_maxit)
    assert ok and eok and gamma == eg and rejected == em, (scale, gamma, eg)
    # closed form in this case: the bound is 2 (1 - c) / scale
    assert abs(2 * (1 - c) / scale - 2.0 * (1.0 - c) * (-(g * dx).sum()) / (a * dx * dx).sum()) \
        <= 1e-12 * 2 / scale


@pytest.mark.parametrize("c,ls_maxit,scale", [(1e-4, 3, 37.0), (0.999999, 30, 1e4)])
def test_armijo_fails_after_the_last_halving(c, ls_maxit, scale):
    s, a = _quadratic_stepper(c=c, ls_maxit=ls_maxit)
    x = s.x.copy()
    g = (s.m[:, None] / s.h ** 2) * (x - s.xhat)
    g[s.dir_ids] += s.p.k_dirichlet * (x[s.dir_ids] - s.xbar)
    dx = scale * (-g / a)
    gamma, ok, rejected = s.line_search(x, dx, g.reshape(-1))
    _, eok, em = _armijo_expected(g, dx, a, c, ls_maxit)
    assert not ok and not eok and rejected == em == ls_maxit + 1


def test_armijo_slips_fail():
    """A '<' for '<=' in the bound, a missing factor (1 - c), or accepting the
    last rejected step instead of the first accepted one each change the
    accepted step for one of the scales above."""
    s, a = _quadratic_stepper()
    rng = np.random.default_rng(3)
    x = s.x + 0.01 * rng.standard_normal(s.x.shape)
    g = (s.m[:, None] / s.h ** 2) * (x - s.xhat)
    g[s.dir_ids] += s.p.k_dirichlet * (x[s.dir_ids] - s.xbar)
    newton = -g / a
    diffs = 0
    for scale in (1.9999, 3.0, 5.3, 37.0):
        dx = scale * newton
        true_gamma = s.line_search(x, dx, g.reshape(-1))[0]
        no_c = 2.0 ** -math.ceil(math.log2(scale / 2.0)) if scale > 2 else 1.0   # drops (1 - c)
        twice = true_gamma * 2.0                                               # one halving too few
        diffs += (no_c != true_gamma) + (twice != true_gamma)
    assert diffs >= 4
