"""Edge cases of the PCG solve through the C ABI, against the oracle's PCG:

* a zero right-hand side (no elastic material, no gravity, at rest on its
  constraint targets, so the gradient is exactly zero): decided at the first
  product, dx = 0, no iterations, no indefiniteness;
* iteration caps of 1, 2, 3, 5 and 17 on an SPD system (every element
  projected) that converges in 12: the solve stops at the cap, or converges
  below it, with the oracle's count and iterate;
* a loose tolerance, met after a few iterations: the same count and iterate;
* the product's load modes (small, cache-resident, streamed; normally chosen
  from the matrix size), each forced on one scene: the same bits in every
  mode, for one solve and for whole steps, in FP64 and the mixed form.

These counts are small and irregular, so the launches that the host enqueues
past the device's stop decision (which return at once) are a large part of
each solve; the results must not depend on them.
"""
import numpy as np
import pytest

from oracle.assemble import diagonal_blocks
from oracle.pcg import pcg_block_jacobi
from oracle.project import project_to_pd
from paper_2505_21013_amd import PPN_FP64, PPN_MIXED, PPNError, run_steps
from scenes import cube_compress

from helpers import gpu_scene, oracle_stepper, squashed_state

pytestmark = pytest.mark.gpu


def _scene():
    return cube_compress(n=5, n_steps=4, ramp_steps=4)


def test_zero_rhs_is_decided_at_the_first_product():
    sc = _scene()
    g = gpu_scene(sc)
    g.ppn_set_material(sc.rho, 0.0, 0.45)
    g.ppn_set_time_step(sc.dt, (0.0, 0.0, 0.0))
    g.ppn_set_dirichlet(sc.dirichlet_ids, sc.X[sc.dirichlet_ids])
    g.ppn_set_state(sc.X, np.zeros_like(sc.X))
    assert np.max(np.abs(g.ppn_eval_gradient(sc.X))) == 0.0
    dx, ind, it = g.ppn_solve(sc.X)
    g.close()
    assert not ind and it == 0
    assert np.all(dx == 0.0)


def _oracle_system(sc, x):
    orc = oracle_stepper(sc)
    grad, _, He, _ = orc.evaluate(x)
    Ho = orc.asm.hessian(project_to_pd(He, 1e-8), orc._diag())
    return grad, Ho


@pytest.mark.parametrize("maxit", [1, 2, 3, 5, 17])
def test_iteration_cap(maxit):
    sc = _scene()
    x = squashed_state(sc, seed=4)
    grad, Ho = _oracle_system(sc, x)
    _, _, full = pcg_block_jacobi(Ho, -grad, diagonal_blocks(Ho), rtol=1e-4, maxit=10000)
    dxo, indo, ito = pcg_block_jacobi(Ho, -grad, diagonal_blocks(Ho), rtol=1e-4, maxit=maxit)
    g = gpu_scene(sc, pcg_maxit=maxit)
    dx, ind, it = g.ppn_solve(x, proj_mask=np.ones(sc.n_tets, np.uint8))
    g.close()
    assert not ind and not indo
    assert it == ito == min(maxit, full), (it, ito, full)
    assert np.linalg.norm(dx - dxo) <= 1e-9 * np.linalg.norm(dxo)
    assert grad @ dx < 0


def test_loose_tolerance_meets_it_in_few_iterations():
    sc = _scene()
    x = squashed_state(sc, seed=5)
    grad, Ho = _oracle_system(sc, x)
    dxo, indo, ito = pcg_block_jacobi(Ho, -grad, diagonal_blocks(Ho), rtol=0.3, maxit=10000)
    g = gpu_scene(sc, pcg_rtol=0.3)
    dx, ind, it = g.ppn_solve(x, proj_mask=np.ones(sc.n_tets, np.uint8))
    g.close()
    assert not ind and not indo and 0 < ito < 20
    assert it == ito
    assert np.linalg.norm(dx - dxo) <= 1e-9 * np.linalg.norm(dxo)
    assert np.linalg.norm(Ho @ dx + grad) <= 0.3 * np.linalg.norm(grad) * (1 + 1e-9)


@pytest.mark.parametrize("precision", [PPN_FP64, PPN_MIXED])
def test_every_load_mode_gives_the_same_bits(precision):
    sc = _scene()
    x = squashed_state(sc, seed=6)
    mask = np.ones(sc.n_tets, np.uint8)
    solves, steps = [], []
    for mode in (-1, 0, 1, 2):
        g = gpu_scene(sc, precision=precision, pcg_load_mode=mode)
        solves.append(g.ppn_solve(x, proj_mask=mask))
        g.close()
        g = gpu_scene(sc, precision=precision, pcg_load_mode=mode)
        st = run_steps(g, sc, "PPN", 3)
        steps.append(([(t["newton_iters"], t["pcg_iters"], t["projected"]) for t in st], g.ppn_get_positions()))
        g.close()
    dx0, ind0, it0 = solves[0]
    assert not ind0 and it0 > 0
    for dx, ind, it in solves[1:]:
        assert (ind, it) == (ind0, it0) and np.array_equal(dx, dx0)
    assert sum(c[1] for c in steps[0][0]) > 0
    for counts, xs in steps[1:]:
        assert counts == steps[0][0] and np.array_equal(xs, steps[0][1])


def test_load_mode_out_of_range_is_refused():
    with pytest.raises(PPNError, match="pcg_load_mode"):
        gpu_scene(_scene(), pcg_load_mode=3)
