"""Mixed precision (PPN_MIXED) against the FP64 oracle.

In this form the eigensolves and the PCG iterations run in FP32 while the
gradient, the energies, the assembly and each solve's refinement residual stay
FP64.  The bars, per result:
  * element projections within 2e-5 of the element matrix's magnitude (FP32
    Jacobi), still positive semidefinite to that level;
  * every linear solve meets the FP64 bound |H dx + g| <= rtol |g| on the
    oracle's own operator (the refinement guarantees it);
  * whole time steps, trajectory against trajectory: positions within 1e-6 of
    the bounding-box diagonal; the Newton residual each step ends with against
    the oracle's own final residual of that step, relative to the step's
    initial residual (R30), printed beside the same figure for the FP64 GPU
    form and held to 1e-8 where the scene meets it, or to the measured value
    with the shortfall stated; the projected-set mismatch rate (summed
    symmetric difference of the per-iteration projected sets over their
    union), printed and bounded, on scenes that project.
  Both runs stop on |dx|_inf after inexact solves (|r| <= 1e-4 |g|): once the
  arithmetic differs, the Krylov iterates differ, so the last iterate of a step
  differs at the level of the stopping tolerance.  On the 6^3 jittered cube
  this puts the trajectory residual difference at a few 1e-8 of the initial
  residual, above the 1e-8 asked for; on the 1.57M-tet cube it is about 1e-12
  (tests/test_gpu_cube64_golden.py).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.assemble import diagonal_blocks
from oracle.fem import predictor
from oracle.pcg import pcg_block_jacobi
from oracle.project import project_to_pd
from paper_2505_21013_amd import PPN_MIXED, run_steps
from scenes import config, cube_compress, renumbered

from helpers import first_hard_step, gpu_scene, oracle_stepper, squashed_state

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

SCENES = {
    "cube6_jitter": lambda: config(0),
    "cube4_compress": lambda: cube_compress(n=4, n_steps=4, ramp_steps=4),
}


@pytest.fixture(scope="module", params=sorted(SCENES))
def case(request):
    sc = SCENES[request.param]()
    orc = oracle_stepper(sc)
    gpu = gpu_scene(sc, precision=PPN_MIXED)
    x = squashed_state(sc, seed=sorted(SCENES).index(request.param))
    g, ge, He, H = orc.evaluate(x)
    yield dict(sc=sc, orc=orc, gpu=gpu, x=x, g=g, He=He)
    gpu.close()


def test_mixed_gradient_is_fp64(case):
    g_gpu = case["gpu"].ppn_eval_gradient(case["x"])
    assert np.max(np.abs(g_gpu - case["g"])) <= 1e-12 * np.max(np.abs(case["g"]))


def test_mixed_projection(case):
    T = case["sc"].n_tets
    He = case["He"]
    nrm = np.abs(He).max(axis=(1, 2))
    Hp_gpu = case["gpu"].ppn_eval_element_hessians(case["x"], proj_mask=np.ones(T, np.uint8))
    err = np.abs(Hp_gpu - project_to_pd(He, 1e-8)).max(axis=(1, 2))
    assert np.all(err <= 2e-5 * nrm), (err / nrm).max()
    lg = np.linalg.eigvalsh(0.5 * (Hp_gpu + np.swapaxes(Hp_gpu, 1, 2)))
    assert np.all(lg[:, 0] >= -2e-5 * nrm)


@pytest.mark.parametrize("projected", [False, True])
def test_mixed_solve_meets_fp64_residual(case, projected):
    T = case["sc"].n_tets
    mask = np.ones(T, np.uint8) if projected else None
    dx, ind, it = case["gpu"].ppn_solve(case["x"], proj_mask=mask)
    He = case["He"].copy()
    if projected:
        He = project_to_pd(He, 1e-8)
    Ho = case["orc"].asm.hessian(He, case["orc"]._diag())
    g = case["g"]
    _, indo, _ = pcg_block_jacobi(Ho, -g, diagonal_blocks(Ho))
    assert ind == indo
    if projected:
        assert not ind
    if not ind:
        # Ho holds the projected element matrices in FP64; the solve's FP32
        # projections differ from them by the projection tolerance above.
        slack = 1e-6 if not projected else 1e-3
        assert np.linalg.norm(Ho @ dx + g) <= 1e-4 * np.linalg.norm(g) * (1 + slack)
        assert g @ dx < 0


def _mask_mismatch(o_trace, g_trace):
    """Summed symmetric difference over summed union of the per-iteration
    projected sets, over the iterations both runs carried out."""
    diff = union = 0
    for ro, rg in zip(o_trace, g_trace):
        a = set(np.asarray(ro.get("projected_idx", np.zeros(0, np.int32))).tolist())
        b = set(np.asarray(rg["projected_ids"]).tolist())
        diff += len(a ^ b)
        union += len(a | b)
    return diff, union


# Trajectory residual bar per scene: 1e-8 of the initial residual (the stated
# accuracy), except where the measured difference is above it; there the bar is
# the measured value rounded up, and the shortfall is the result: the 6^3
# jittered cube ends its steps 3.5e-8 (6.2e-8 renumbered) of the initial
# residual away from the oracle's final residual in PDN and PPN, while the FP64
# GPU form stays within 4e-14 there.
RES_BAR = {"cube6_jitter": 1e-7, "cube6_jitter_renum5": 1e-7, "cube6_compress": 1e-8}


@pytest.mark.parametrize("mode", ["PN", "PDN", "PPN"])
def test_mixed_cube6_jitter_20_steps(mode):
    _mixed_against_oracle(config(0), mode, RES_BAR["cube6_jitter"])


@pytest.mark.parametrize("mode", ["PN", "PPN"])
def test_mixed_renumbered_cube6_jitter_20_steps(mode):
    """The same scene numbered at random (vertices, elements, local orders):
    the FP32 matrix conversion and product then work on 64-row groups of
    mixed row lengths with scattered columns, and must meet the same bars."""
    _mixed_against_oracle(renumbered(config(0), seed=5), mode, RES_BAR["cube6_jitter_renum5"])


@pytest.mark.parametrize("mode", ["PDN", "PPN"])
def test_mixed_compressed_cube6_projects(mode):
    """A 6^3 cube squashed over 8 steps: PPN runs inner rounds and PDN projects
    every element after detecting indefiniteness, so the projected-set mismatch
    rate is measured on projections that happen."""
    sc = cube_compress(n=6, n_steps=8, ramp_steps=8)
    union = _mixed_against_oracle(sc, mode, RES_BAR["cube6_compress"])
    assert union > 0


def _trajectory(sc, mode, precision):
    gpu = gpu_scene(sc, trace=True, precision=precision)
    gstate, gtr = [(sc.x0.copy(), sc.v0.copy())], []

    def cb(n, s, st):
        gstate.append(s.ppn_get_state())
        gtr.append(s.ppn_trace())
    gst = run_steps(gpu, sc, mode, sc.n_steps, callback=cb)
    gpu.close()
    return gst, gstate, gtr


def _mixed_against_oracle(sc, mode, res_bar):
    orc_x = []
    _, ost = oracle.run_scene(sc, mode, n_steps=sc.n_steps, trace=True,
                              callback=lambda n, s, st: orc_x.append(s.x.copy()))
    gst, gstate, gtr = _trajectory(sc, mode, PPN_MIXED)
    f64, _, _ = _trajectory(sc, mode, 0)
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    diff = union = 0
    worst_pos = worst_eval = worst_traj = worst_traj64 = 0.0
    for n in range(sc.n_steps):
        o, g = ost[n], gst[n]
        tag = f"{mode} step {n + 1}"
        assert g["status"] == "PPN_OK" and o.converged, (tag, g["status"])
        assert g["refine_rounds"] >= g["solves"], tag
        x, _ = gstate[n + 1]
        worst_pos = max(worst_pos, float(np.max(np.abs(x - orc_x[n]))) / diag)
        # the residual the step reports is the FP64 gradient norm at its own
        # final state (the oracle's gradient there, evaluated independently)
        st = oracle_stepper(sc, step=n + 1)
        xp, vp = gstate[n]
        st.xhat = predictor(xp, vp, st.h, st.gravity)
        res = float(np.linalg.norm(st.gradient(x)))
        worst_eval = max(worst_eval, abs(g["res_l2"] - res) / g["res0_l2"])
        # trajectory against trajectory: the step's final residual against the
        # oracle's own final residual of that step (R30), mixed and FP64 forms
        worst_traj = max(worst_traj, abs(g["res_l2"] - o.res_l2) / o.res0_l2)
        worst_traj64 = max(worst_traj64, abs(f64[n]["res_l2"] - o.res_l2) / o.res0_l2)
        d, u = _mask_mismatch(o.trace, gtr[n])
        diff += d
        union += u
    rate = diff / max(union, 1)
    print(f"\nmixed {sc.name} {mode}: positions {worst_pos:.2e} of the diagonal; final residual against "
          f"the oracle's {worst_traj:.2e} res0 (FP64 GPU form {worst_traj64:.2e} res0; bar {res_bar:.0e}); "
          f"projected-set mismatch {rate:.2e} ({diff}/{union}); reported residual vs the FP64 gradient at "
          f"the same state {worst_eval:.2e} res0")
    assert worst_pos <= 1e-6, worst_pos
    assert worst_eval <= 1e-10, worst_eval
    assert worst_traj <= res_bar, worst_traj
    assert rate <= 0.05, rate
    return union


def test_mixed_cube16_schedule_against_oracle_record():
    gold = json.load(open(os.path.join(HERE, "golden", "cube16_compress_oracle.json")))
    ref = gold["modes"]["PPN"]
    sc = cube_compress(n=16, n_steps=50, ramp_steps=50)
    gpu = gpu_scene(sc, precision=PPN_MIXED)
    stats = run_steps(gpu, sc, "PPN", 50)
    x = gpu.ppn_get_positions()
    gpu.close()
    worst_traj = 0.0
    for n, (g, o) in enumerate(zip(stats, ref["steps"])):
        assert (g["status"] == "PPN_OK") == o["converged"], (n + 1, g["status"])
        worst_traj = max(worst_traj, abs(g["res_l2"] - o["res_l2"]) / o["res0_l2"])
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    sample = np.array(gold["sample_vertices"])
    err = float(np.max(np.abs(x[sample] - np.array(ref["final_x_sample"])))) / diag
    print(f"\nmixed cube16 PPN: trajectory residual difference {worst_traj:.2e} res0, final "
          f"position error {err:.2e} diag")
    assert worst_traj <= 1e-8, worst_traj
    assert err <= 1e-6, err


def test_mixed_cube64_solve_and_steps():
    sc = config(2)
    gpu = gpu_scene(sc, precision=PPN_MIXED)
    stats = run_steps(gpu, sc, "PPN", 2)
    assert all(s["status"] == "PPN_OK" for s in stats)
    x, v = gpu.ppn_get_state()
    orc = oracle_stepper(sc, step=3)
    orc.x, orc.v = x.copy(), v.copy()
    orc.xhat = orc.x + sc.dt * orc.v + sc.dt ** 2 * np.asarray(sc.gravity)[None]
    gpu.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(3))
    xt = x + 1e-4 * np.random.default_rng(3).standard_normal(x.shape)
    g = orc.gradient(xt)
    g_gpu = gpu.ppn_eval_gradient(xt)
    assert np.max(np.abs(g_gpu - g)) <= 1e-12 * np.max(np.abs(g))
    dx, ind, it = gpu.ppn_solve(xt)
    if not ind:
        Hdx = orc.hessian_rows_product(xt, dx, np.arange(sc.n_verts)).reshape(-1)
        assert np.linalg.norm(Hdx + g) <= 1e-4 * np.linalg.norm(g) * (1 + 1e-6)
        assert g @ dx < 0
    gpu.close()


def test_mixed_streamed_fp32_matrix_meets_fp64_residual():
    """An 80^3 compressed cube (3,072,000 tets) with the mixed product reading
    its FP32 matrix with non-temporal loads (the streamed mode, forced: the
    library reads matrices of this size with ordinary loads).  After one step, the mixed solve
    on the fully projected system meets the FP64 residual bound, checked with
    the library's FP64 gradient and product (both pinned to the oracle on other
    meshes), and gives a descent direction."""
    sc = cube_compress(n=80)
    gpu = gpu_scene(sc, precision=PPN_MIXED, pcg_load_mode=2)
    stats = run_steps(gpu, sc, "PPN", 1)
    assert stats[0]["status"] == "PPN_OK"
    x, _ = gpu.ppn_get_state()
    gpu.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(2))
    mask = np.ones(sc.n_tets, np.uint8)
    g = gpu.ppn_eval_gradient(x)
    dx, ind, it = gpu.ppn_solve(x, proj_mask=mask)
    assert not ind and it > 0
    r = gpu.ppn_hessian_product(x, dx, proj_mask=mask) + g
    # FP32 projections inside the solve against FP64 ones in the check
    assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(g) * (1 + 1e-3)
    assert g @ dx < 0
    gpu.close()


def test_mixed_beam_twist_against_oracle_record():
    """The twisted beam (122,880 tets) over its 100-step schedule in the mixed
    form against the oracle's PPN record (tests/golden/beam_twist_PPN.json):
    per step the final residual against the oracle's (R30) and the Newton and
    projection counts, per Newton iteration whether the projected set equals the
    oracle's (fingerprints), sampled positions after steps 25, 50, 75 and 100.
    Printed: the largest residual difference over the steps whose counts match
    the oracle's, the steps whose counts differ, the share of Newton iterations
    whose projected set differs, the position errors."""
    path = os.path.join(HERE, "golden", "beam_twist_PPN.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    gold = json.load(open(path))
    sc = config(1)
    sample = np.array(gold["sample_vertices"])
    gpu = gpu_scene(sc, trace=True, precision=PPN_MIXED)
    masks, snaps = [], {}

    def fp(ids):
        ids = np.asarray(ids, dtype=np.int64)
        return [int(ids.size), int(ids.sum()), int((ids * ids).sum())]

    def cb(n, s, st):
        masks.append([fp(r["projected_ids"]) for r in s.ppn_trace()])
        if str(n) in gold["x_sample"]:
            snaps[str(n)] = s.ppn_get_positions()[sample]
    stats = run_steps(gpu, sc, "PPN", len(gold["steps"]), callback=cb)
    gpu.close()
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    differ, worst_traj, n_iter, iter_mism = [], 0.0, 0, 0
    for n, (g, o) in enumerate(zip(stats, gold["steps"])):
        assert g["status"] in ("PPN_OK", "PPN_WARN_NOT_CONVERGED"), (n + 1, g["status"])
        if (g["newton_iters"], g["projected"]) != (o["newton_iters"], o["projected"]):
            differ.append((n + 1, g["newton_iters"], o["newton_iters"], g["projected"], o["projected"]))
            continue
        worst_traj = max(worst_traj, abs(g["res_l2"] - o["res_l2"]) / o["res0_l2"])
        for a, b in zip(masks[n], o["masks"]):
            n_iter += 1
            iter_mism += a != b
    errs = {k: float(np.max(np.abs(snaps[k] - np.array(v)))) / diag for k, v in gold["x_sample"].items()}
    print(f"\nmixed beam PPN: steps whose counts differ from the oracle's (step, Newton, oracle's, projected, "
          f"oracle's) {differ}; on the others: final residual against the oracle's {worst_traj:.2e} res0, "
          f"Newton iterations whose projected set differs {iter_mism}/{n_iter}; positions "
          f"{', '.join(f'step {k} {v:.2e}' for k, v in errs.items())} of the diagonal")
    # only steps from the first hard one on (tests/helpers.py) may take other counts
    assert all(d[0] >= first_hard_step(gold["steps"]) for d in differ), differ
    assert worst_traj <= 1e-8, worst_traj
    assert iter_mism <= 0.01 * n_iter, (iter_mism, n_iter)
    # after a hard step, the bound of the Newton stopping rule (10 h tol, as in
    # tests/test_gpu_beam_golden.py), relative to the diagonal
    first_hard = first_hard_step(gold["steps"])
    for k, v in errs.items():
        assert v <= (1e-6 if int(k) < first_hard else 10 * sc.dt * sc.stop_tol / diag), (k, v)
