"""Per-stage parity of the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded synthetic scenes; sizes span several 256-wide workgroups
with a ragged tail (cube 6^3: 1296 tets = 5*256 + 16; cube 4^3: 384 tets).
Tolerances are relative to the magnitude of the quantity compared; the
selection mask, which is an integer decision taken in FP64 on both sides from
the same assembled gradient, must be bit-exact.
"""
import numpy as np
import pytest

from oracle.project import project_to_pd
from oracle.pcg import pcg_block_jacobi
from oracle.assemble import diagonal_blocks
from scenes import beam_twist, config, cube_compress

from helpers import bsr_to_csr, gpu_scene, oracle_stepper, squashed_state

pytestmark = pytest.mark.gpu

SCENES = {
    "cube6_jitter": lambda: config(0),
    "cube4_compress": lambda: cube_compress(n=4, n_steps=4, ramp_steps=4),
    "beam10_twist": lambda: beam_twist(nx=10, ny=2, nz=3, L=0.25, W=0.05, n_steps=8, turns=0.5),
}


@pytest.fixture(scope="module", params=sorted(SCENES))
def case(request):
    sc = SCENES[request.param]()
    orc = oracle_stepper(sc)
    gpu = gpu_scene(sc)
    x = squashed_state(sc, seed=sorted(SCENES).index(request.param))
    g, ge, He, H = orc.evaluate(x)
    yield dict(name=request.param, sc=sc, orc=orc, gpu=gpu, x=x, g=g, He=He, H=H)
    gpu.close()


def test_gradient(case):
    g_gpu = case["gpu"].ppn_eval_gradient(case["x"])
    g = case["g"]
    assert np.max(np.abs(g_gpu - g)) <= 1e-12 * np.max(np.abs(g))


def test_element_hessians(case):
    He_gpu = case["gpu"].ppn_eval_element_hessians(case["x"])
    He = case["He"]
    scale = np.abs(He).max(axis=(1, 2))
    err = np.abs(He_gpu - He).max(axis=(1, 2))
    assert np.all(err <= 1e-12 * scale), err.max() / scale[np.argmax(err / scale)]


def test_element_projection(case):
    T = case["sc"].n_tets
    He = case["He"]
    lam = np.linalg.eigvalsh(He)
    nrm = np.abs(He).max(axis=(1, 2))
    assert np.any(lam[:, 0] < -1e-6 * nrm), "state must contain indefinite elements"
    Hp_gpu = case["gpu"].ppn_eval_element_hessians(case["x"], proj_mask=np.ones(T, np.uint8))
    Hp = project_to_pd(He, 1e-8)
    err = np.abs(Hp_gpu - Hp).max(axis=(1, 2))
    assert np.all(err <= 1e-11 * nrm), (err / nrm).max()
    lg = np.linalg.eigvalsh(0.5 * (Hp_gpu + np.swapaxes(Hp_gpu, 1, 2)))
    assert np.all(lg[:, 0] >= 1e-8 - 1e-12 * nrm)


def test_assembled_hessian_and_pattern(case):
    n = case["sc"].n_verts
    T = case["sc"].n_tets
    rng = np.random.default_rng(3)
    mask = (rng.uniform(size=T) < 0.3).astype(np.uint8)
    rp, col, vals = case["gpu"].ppn_eval_hessian(case["x"], proj_mask=mask)
    Hg = bsr_to_csr(rp, col, vals, n)
    orc = case["orc"]
    He = case["He"].copy()
    sel = mask.astype(bool)
    He[sel] = project_to_pd(He[sel], 1e-8)
    Ho = orc.asm.hessian(He, orc._diag())
    D = (Hg - Ho).tocsr()
    assert abs(D).max() <= 1e-11 * abs(Ho).max()
    # block pattern: exactly the vertex pairs that share an element, plus the diagonal
    Hb = Ho.tobsr(blocksize=(3, 3))
    Hb.sort_indices()
    assert np.array_equal(Hb.indptr, rp) and np.array_equal(Hb.indices, col)


def test_selection_is_bit_exact(case):
    sc, orc = case["sc"], case["orc"]
    T = sc.n_tets
    rng = np.random.default_rng(11)
    g = case["g"] * rng.lognormal(0, 1.0, size=case["g"].shape)
    s_e = orc.selection_residual(g)
    ginf = np.abs(g).max()
    deltas = [0.5 * ginf, 0.125 * ginf, 2.0 ** -10 * ginf, float(np.median(s_e)), float(s_e[7]),
              1e-13, 0.0, 2.0 * ginf]
    for trial, delta in enumerate(deltas):
        proj_in = (rng.uniform(size=T) < 0.2 * (trial % 2)).astype(np.uint8)
        expect = (proj_in == 0) & ((s_e > delta) | (delta <= 1e-12))
        mask, cnt = case["gpu"].ppn_select(g, delta, proj_in)
        assert np.array_equal(mask.astype(bool), expect), (delta, np.sum(mask != expect))
        assert cnt == int(expect.sum())


def test_hessian_product(case):
    n = case["sc"].n_verts
    T = case["sc"].n_tets
    rng = np.random.default_rng(5)
    d = rng.standard_normal(3 * n)
    mask = (rng.uniform(size=T) < 0.5).astype(np.uint8)
    q = case["gpu"].ppn_hessian_product(case["x"], d, proj_mask=mask)
    He = case["He"].copy()
    sel = mask.astype(bool)
    He[sel] = project_to_pd(He[sel], 1e-8)
    Ho = case["orc"].asm.hessian(He, case["orc"]._diag())
    qo = Ho @ d
    assert np.max(np.abs(q - qo)) <= 1e-12 * np.max(np.abs(qo))


@pytest.mark.parametrize("projected", [False, True])
def test_pcg(case, projected):
    T = case["sc"].n_tets
    mask = np.ones(T, np.uint8) if projected else None
    dx, ind, it = case["gpu"].ppn_solve(case["x"], proj_mask=mask)
    He = case["He"].copy()
    if projected:
        He = project_to_pd(He, 1e-8)
    Ho = case["orc"].asm.hessian(He, case["orc"]._diag())
    g = case["g"]
    dxo, indo, ito = pcg_block_jacobi(Ho, -g, diagonal_blocks(Ho))
    assert ind == indo
    assert abs(it - ito) <= 1, (it, ito)
    if projected:
        assert not ind
    if not ind:
        assert np.linalg.norm(Ho @ dx + g) <= 1e-4 * np.linalg.norm(g) * (1 + 1e-6)
        assert g @ dx < 0
    if it == ito:
        assert np.linalg.norm(dx - dxo) <= 1e-6 * max(np.linalg.norm(dxo), 1e-300)


def test_energy_difference(case):
    n = case["sc"].n_verts
    rng = np.random.default_rng(9)
    dx = 0.01 * rng.standard_normal((n, 3)) * np.ptp(case["sc"].X) / max(case["sc"].meta["cells"])
    gam = np.array([1.0, 0.5, 0.25, 0.125, 2.0 ** -10])
    out = case["gpu"].ppn_energy_difference(case["x"], dx, gam)
    ref = np.array([case["orc"].energy_difference(case["x"], dx, g) for g in gam])
    scale = np.abs(ref).max()
    assert np.all(np.abs(out - ref) <= 1e-10 * scale + 1e-12 * np.abs(ref))


def test_project_batch_known_spectra():
    """Stateless batch projector on matrices with a translation null space and
    prescribed spectra, including the eigenvalues of the paper's worked
    example (-1, 2, -10, 1)."""
    torch = pytest.importorskip("torch")
    from paper_2505_21013_amd import ppn_project_batch_dev
    rng = np.random.default_rng(2)
    n = 777
    # orthonormal complement of the translations: U = 1/2 Had4 (x) I3, rows 3..11
    had = 0.5 * np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], float)
    U = np.kron(had, np.eye(3))
    Hs = np.empty((n, 12, 12))
    for k in range(n):
        Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
        lam = rng.uniform(-5, 50, 9) * 10 ** rng.uniform(-2, 3)
        if k == 0:
            lam = np.array([-1.0, 2.0, -10.0, 1.0, 2.0, 2.0, 5.0, 7.0, 9.0])
        K = Q @ np.diag(lam) @ Q.T
        Z = np.zeros((12, 12))
        Z[3:, 3:] = K
        Hs[k] = U @ Z @ U
        Hs[k] = 0.5 * (Hs[k] + Hs[k].T)
    dev = torch.from_numpy(Hs.reshape(-1)).cuda()
    out = torch.empty_like(dev)
    ppn_project_batch_dev(dev, out, n, 1e-8)
    got = out.cpu().numpy().reshape(n, 12, 12)
    ref = project_to_pd(Hs, 1e-8)
    nrm = np.abs(Hs).max(axis=(1, 2))
    assert np.all(np.abs(got - ref).max(axis=(1, 2)) <= 1e-11 * nrm)
    ev = np.linalg.eigvalsh(got[0])
    assert np.allclose(ev[3:], sorted([1e-8, 2.0, 1e-8, 1.0, 2.0, 2.0, 5.0, 7.0, 9.0]), atol=1e-12)
    # in place (aliased input and output)
    ppn_project_batch_dev(dev, dev, n, 1e-8)
    assert np.array_equal(dev.cpu().numpy().reshape(n, 12, 12), got)


def test_project_batch_rejects_matrices_outside_its_precondition():
    """The dense projector deflates the rigid translations exactly, so it takes
    only symmetric matrices that annihilate them: -I, an asymmetric element
    Hessian and a NaN entry are each refused with PPN_ERR_ARG, and nothing is
    written (the output keeps its sentinel values)."""
    torch = pytest.importorskip("torch")
    from paper_2505_21013_amd import PPNError, ppn_project_batch_dev
    had = 0.5 * np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], float)
    U = np.kron(had, np.eye(3))
    Z = np.zeros((12, 12))
    Z[3:, 3:] = np.diag(np.arange(-4.0, 5.0))
    good = U @ Z @ U
    good = 0.5 * (good + good.T)
    asym = good.copy()
    asym[3, 7] += 1e-3 * np.abs(good).max()
    nan = good.copy()
    nan[5, 5] = np.nan
    for bad in (-np.eye(12), asym, nan):
        Hs = np.stack([good, bad, good])
        dev = torch.from_numpy(Hs.reshape(-1)).cuda()
        out = torch.full_like(dev, 7.0)
        with pytest.raises(PPNError) as ei:
            ppn_project_batch_dev(dev, out, 3, 1e-8)
        assert ei.value.code == -1
        assert torch.all(out == 7.0).item()
        # aliased: the input is left untouched too
        with pytest.raises(PPNError):
            ppn_project_batch_dev(dev, dev, 3, 1e-8)
        assert np.array_equal(dev.cpu().numpy(), Hs.reshape(-1), equal_nan=True)
    ok = torch.from_numpy(np.stack([good] * 3).reshape(-1)).cuda()
    ppn_project_batch_dev(ok, ok, 3, 1e-8)
    assert np.linalg.eigvalsh(ok.cpu().numpy().reshape(3, 12, 12)[0]).min() >= 1e-8 - 1e-12
