"""Pins of the FP64 CPU oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against mathematics the paper or the
material model fixes: finite differences, closed forms, invariances, the
paper's worked example, dense linear algebra on tiny meshes and invariants of
Algorithm 1.  A plausible slip in the oracle (a dropped term, a sign, a
transposed operand, a wrong index) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import snh
from oracle.assemble import Assembler, diagonal_blocks
from oracle.fem import Mesh, element_grad_hess, element_psi, lumped_mass
from oracle.newton import Params, Stepper, run_scene
from oracle.pcg import pcg_block_jacobi
from oracle.project import project_to_pd
from scenes import beam_twist, config, cube_compress, kuhn_grid

HERE = os.path.dirname(os.path.abspath(__file__))
MU, LAM = snh.lame_to_snh(1e5, 0.45)


def random_F(rng, n, spread=0.4, allow_inverted=True):
    F = np.eye(3)[None] + spread * rng.standard_normal((n, 3, 3))
    if allow_inverted:
        F[: n // 4, :, 0] *= -1.0  # some with J < 0
    return F


# ---------------------------------------------------------------- P1: finite differences
def test_P1_psi_to_P_finite_differences():
    rng = np.random.default_rng(1)
    F = random_F(rng, 16)
    P = snh.first_piola(F, MU, LAM)
    h = 1e-6
    for t in range(F.shape[0]):
        fd = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                E = np.zeros((3, 3)); E[i, j] = h
                fd[i, j] = (snh.psi(F[t] + E, MU, LAM) - snh.psi(F[t] - E, MU, LAM)) / (2 * h)
        assert np.max(np.abs(fd - P[t])) <= 1e-7 * max(1.0, np.max(np.abs(P[t])))


def test_P1_P_to_A_finite_differences():
    rng = np.random.default_rng(2)
    F = random_F(rng, 16)
    A = snh.d2psi_dF2(F, MU, LAM)
    h = 1e-6
    for t in range(F.shape[0]):
        fd = np.zeros((9, 9))
        for l in range(9):
            E = np.zeros(9); E[l] = h
            Em = E.reshape(3, 3).T  # vec index 3j+i -> F[i, j]
            fd[:, l] = (snh.vec(snh.first_piola(F[t] + Em, MU, LAM))
                        - snh.vec(snh.first_piola(F[t] - Em, MU, LAM))) / (2 * h)
        assert np.max(np.abs(fd - A[t])) <= 1e-7 * max(1.0, np.max(np.abs(A[t])))
        assert np.allclose(A[t], A[t].T, rtol=0, atol=1e-9 * np.abs(A[t]).max())


def _one_tet_mesh(rng, E=1e5, nu=0.45):
    X = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.1]], float) + 0.01 * rng.standard_normal((4, 3))
    tets = np.array([[0, 1, 2, 3]])
    if np.linalg.det((X[1:] - X[0]).T) < 0:
        tets = np.array([[0, 2, 1, 3]])
    return Mesh.build(X, tets, E, nu)


def test_P1_element_energy_gradient_hessian_finite_differences():
    rng = np.random.default_rng(3)
    for trial in range(6):
        mesh = _one_tet_mesh(rng)
        x = mesh.X + 0.03 * rng.standard_normal(mesh.X.shape)
        if trial % 2:
            x[3] = x[0] - (x[3] - x[0])  # inverted element
        g, H = element_grad_hess(mesh, x)
        h = 1e-7
        fd_g = np.zeros(12)
        fd_H = np.zeros((12, 12))
        for p in range(12):
            dx = np.zeros(12); dx[p] = h
            xp, xm = x + dx.reshape(4, 3), x - dx.reshape(4, 3)
            fd_g[p] = (element_psi(mesh, xp)[0] - element_psi(mesh, xm)[0]) / (2 * h)
            fd_H[:, p] = (element_grad_hess(mesh, xp)[0][0] - element_grad_hess(mesh, xm)[0][0]) / (2 * h)
        assert np.max(np.abs(fd_g - g[0])) <= 1e-7 * np.max(np.abs(g[0]))
        assert np.max(np.abs(fd_H - H[0])) <= 1e-6 * np.max(np.abs(H[0]))


# ---------------------------------------------------------------- P2: rest state
def test_P2_rest_state_zero_stress():
    P = snh.first_piola(np.eye(3)[None], MU, LAM)
    assert np.all(P == 0.0)
    assert snh.psi(np.eye(3)[None], MU, LAM)[0] == 0.0
    X, tets = kuhn_grid(2, 2, 2)
    mesh = Mesh.build(X, tets, 1e5, 0.45)
    g, _ = element_grad_hess(mesh, X)
    scale = np.max(mesh.V) * MU * np.max(np.abs(mesh.Bm))
    assert np.max(np.abs(g)) <= 1e-13 * scale


# ---------------------------------------------------------------- P3: rotation invariance
def _rotation(rng):
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def test_P3_rotation_invariance():
    rng = np.random.default_rng(4)
    F = random_F(rng, 8)
    Rm = _rotation(rng)
    p0 = snh.psi(F, MU, LAM)
    p1 = snh.psi(Rm[None] @ F, MU, LAM)
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * np.max(np.abs(p0))
    mesh = _one_tet_mesh(rng)
    x = mesh.X + 0.02 * rng.standard_normal((4, 3))
    g0, H0 = element_grad_hess(mesh, x)
    g1, H1 = element_grad_hess(mesh, x @ Rm.T)
    big = np.kron(np.eye(4), Rm)
    assert np.max(np.abs(g1[0] - big @ g0[0])) <= 1e-12 * np.max(np.abs(g0))
    assert np.max(np.abs(H1[0] - big @ H0[0] @ big.T)) <= 1e-12 * np.max(np.abs(H0))


# ---------------------------------------------------------------- P4: textbook rest tangent
def test_P4_rest_tangent_is_linear_elasticity():
    E, nu = 1e5, 0.45
    mu_l = E / (2 * (1 + nu))
    lam_l = E * nu / ((1 + nu) * (1 - 2 * nu))
    A = snh.d2psi_dF2(np.eye(3)[None], *snh.lame_to_snh(E, nu))[0]
    C = np.zeros((9, 9))
    d = np.eye(3)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[3 * j + i, 3 * l + k] = mu_l * (d[i, k] * d[j, l] + d[i, l] * d[j, k]) + lam_l * d[i, j] * d[k, l]
    assert np.max(np.abs(A - C)) <= 1e-13 * np.max(np.abs(C))

    # Element level: the standard linear tetrahedron stiffness V Bv^T D Bv (Voigt notation).
    rng = np.random.default_rng(5)
    mesh = _one_tet_mesh(rng, E, nu)
    _, H = element_grad_hess(mesh, mesh.X)
    Dm = (mesh.X[1:] - mesh.X[0]).T
    grads = np.vstack([-np.linalg.inv(Dm).sum(axis=0), np.linalg.inv(Dm)])  # dN_a/dX
    Bv = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = grads[a]
        Bv[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz], [gy, gx, 0], [0, gz, gy], [gz, 0, gx]]
    Dv = np.zeros((6, 6))
    Dv[:3, :3] = lam_l
    Dv[np.arange(3), np.arange(3)] += 2 * mu_l
    Dv[np.arange(3, 6), np.arange(3, 6)] = mu_l
    K = abs(np.linalg.det(Dm)) / 6 * Bv.T @ Dv @ Bv
    assert np.max(np.abs(H[0] - K)) <= 1e-12 * np.max(np.abs(K))


# ---------------------------------------------------------------- P5: translations are null
def test_P5_translation_null_space():
    rng = np.random.default_rng(6)
    X, tets = kuhn_grid(2, 1, 1)
    mesh = Mesh.build(X, tets, 1e5, 0.45)
    x = X + 0.05 * rng.standard_normal(X.shape)
    _, H = element_grad_hess(mesh, x)
    for c in range(3):
        t = np.zeros(12); t[c::3] = 1.0
        assert np.max(np.abs(H @ t)) <= 1e-14 * np.max(np.abs(H))


# ---------------------------------------------------------------- P6: analytic eigensystem
def test_P6_closed_form_spectrum_at_diagonal_F():
    rng = np.random.default_rng(7)
    for _ in range(5):
        sig = rng.uniform(0.3, 1.6, 3) * rng.choice([1, -1], 3)
        F = np.diag(sig)
        A = snh.d2psi_dF2(F[None], MU, LAM)[0]
        J = np.prod(sig)
        s = LAM * (J - 1) - MU
        ev = [MU + s * sig[k] for k in range(3)] + [MU - s * sig[k] for k in range(3)]
        gv = np.array([sig[1] * sig[2], sig[0] * sig[2], sig[0] * sig[1]])
        M3 = MU * np.eye(3) + LAM * np.outer(gv, gv) + s * np.array([[0, sig[2], sig[1]], [sig[2], 0, sig[0]], [sig[1], sig[0], 0]])
        ev += list(np.linalg.eigvalsh(M3))
        got = np.linalg.eigvalsh(A)
        assert np.max(np.abs(np.sort(ev) - got)) <= 1e-12 * np.max(np.abs(got))


# ---------------------------------------------------------------- P7/P8: projection
def test_P7_P8_projection_properties():
    rng = np.random.default_rng(8)
    X, tets = kuhn_grid(2, 2, 1)
    mesh = Mesh.build(X, tets, 1e5, 0.45)
    x = X.copy()
    x[:, 2] *= 0.3  # strongly compressed: indefinite element Hessians
    x += 0.02 * rng.standard_normal(x.shape)
    _, H = element_grad_hess(mesh, x)
    eps = 1e-8
    Hh = project_to_pd(H, eps)
    nrm = np.linalg.norm(H, axis=(1, 2))
    lam = np.linalg.eigvalsh(H)
    assert np.any(lam[:, 0] < -1e-3 * nrm), "scene should contain indefinite elements"
    lh = np.linalg.eigvalsh(Hh)
    assert np.all(lh[:, 0] >= eps - 1e-13 * nrm)
    assert np.allclose(Hh, np.swapaxes(Hh, 1, 2), atol=1e-14 * nrm.max())
    # Unchanged part of the spectrum: eigenvalues >= eps survive exactly up to rounding.
    keep = lam >= eps
    assert np.all(np.abs(np.where(keep, lh - lam, 0)) <= 1e-12 * nrm[:, None])
    # A matrix whose spectrum is already >= eps is returned unchanged (up to rounding).
    S = Hh + 1.0 * np.eye(12)
    assert np.max(np.abs(project_to_pd(S, eps) - S)) <= 1e-13 * np.linalg.norm(S, axis=(1, 2)).max()


def test_P7m_mirroring_is_the_matrix_absolute_value():
    """Mirroring replaces every eigenvalue by max(|lambda|, eps).  Where every
    |lambda| >= eps that is the matrix absolute value |H| = (H^2)^(1/2), which
    scipy computes by a Schur-based square root (no eigendecomposition of H);
    on prescribed spectra it is Q diag(max(|d|, eps)) Q^T built by hand."""
    import scipy.linalg
    rng = np.random.default_rng(81)
    for _ in range(5):
        Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
        d = rng.uniform(0.5, 3.0, 12) * rng.choice([-1.0, 1.0], 12)
        H = (Q * d) @ Q.T
        H = 0.5 * (H + H.T)
        Hm = project_to_pd(H, 1e-8, mirror=True)
        ref = np.real(scipy.linalg.sqrtm(H @ H))
        assert np.max(np.abs(Hm - ref)) <= 1e-9
        assert np.max(np.abs(Hm - (Q * np.abs(d)) @ Q.T)) <= 1e-12
    # tiny and zero eigenvalues are lifted to eps, as with clamping
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    d = np.array([-2.0, -1e-12, 0.0, 3e-9, 1.0, 5.0])
    H = (Q * d) @ Q.T
    want = (Q * np.maximum(np.abs(d), 1e-8)) @ Q.T
    assert np.max(np.abs(project_to_pd(0.5 * (H + H.T), 1e-8, mirror=True) - want)) <= 1e-13
    # mirroring and clamping agree on matrices with no eigenvalue below eps
    S = (Q * np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])) @ Q.T
    S = 0.5 * (S + S.T)
    assert np.max(np.abs(project_to_pd(S, 1e-8, mirror=True) - project_to_pd(S, 1e-8))) <= 1e-13


# ---------------------------------------------------------------- P9: the paper's worked example
def _paper_example():
    mats = {}
    with open(os.path.join(HERE, "golden", "paper_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            vals = [float(v) for v in line[1:]]
            mats[line[0]] = (np.array(vals[:4]).reshape(2, 2), np.array(vals[4:]))
    return mats


def test_P9_paper_worked_example():
    m = _paper_example()
    A, B, C = m["A"][0], m["B"][0], m["C"][0]
    for k in ("A", "B", "C"):
        assert np.allclose(np.linalg.eigvalsh(m[k][0]), np.sort(m[k][1]))
    assert np.array_equal(A + B, m["P=A+B"][0]) and np.all(np.linalg.eigvalsh(A + B) > 0)
    assert np.array_equal(A + B + C, m["Q=A+B+C"][0]) and np.linalg.eigvalsh(A + B + C)[0] == -9
    eps = 1e-8
    onlyC = A + B + project_to_pd(C[None], eps)[0]
    assert np.allclose(onlyC, np.diag([1 + eps, 5.0]), rtol=0, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(onlyC) > 0)
    # Projecting A alone is insufficient; clamping A gives diag(eps, 2).
    assert np.allclose(project_to_pd(A[None], eps)[0], np.diag([eps, 2.0]), atol=1e-15)
    assert np.linalg.eigvalsh(project_to_pd(A[None], eps)[0] + B + C)[0] < 0
    # Embedded in a 12x12 block-diagonal tile the projection acts block by block.
    T = np.zeros((12, 12)); T[:2, :2] = C; T[2:, 2:] = np.diag(np.arange(1.0, 11.0))
    Th = project_to_pd(T[None], eps)[0]
    assert np.allclose(Th[:2, :2], np.diag([eps, 1.0]), atol=1e-14)
    assert np.allclose(Th[2:, 2:], T[2:, 2:], atol=1e-13)


# ---------------------------------------------------------------- assembly against FD of the total potential
def _stepper(scene, **kw):
    p = Params(stop_mode=scene.stop_mode, stop_tol=scene.stop_tol, **kw)
    s = Stepper(scene.X, scene.tets, scene.E, scene.nu, scene.rho, scene.dt, scene.gravity,
                scene.dirichlet_ids, p, x0=scene.x0, v0=scene.v0)
    s.set_targets(scene.targets(1))
    s.xhat = s.x + scene.dt * s.v + scene.dt ** 2 * np.asarray(scene.gravity)[None]
    return s


def _total_potential(s, x):
    inert = 0.5 * np.sum(s.m[:, None] / s.h ** 2 * (x - s.xhat) ** 2)
    pen = 0.5 * s.p.k_dirichlet * np.sum((x[s.dir_ids] - s.xbar) ** 2)
    return inert + element_psi(s.mesh, x).sum() + pen


def test_assembled_gradient_and_hessian_match_finite_differences():
    rng = np.random.default_rng(9)
    sc = cube_compress(n=2, n_steps=4, ramp_steps=4)
    s = _stepper(sc)
    x = s.x + 0.01 * rng.standard_normal(s.x.shape)
    g, _, _, H = s.evaluate(x)
    h = 1e-7
    for p in rng.choice(g.size, 12, replace=False):
        e = np.zeros(g.size); e[p] = h
        fd = (_total_potential(s, x + e.reshape(-1, 3)) - _total_potential(s, x - e.reshape(-1, 3))) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * np.abs(g).max()
    v = rng.standard_normal(g.size)
    t = 1e-6
    fd = (s.evaluate(x + t * v.reshape(-1, 3))[0] - s.evaluate(x - t * v.reshape(-1, 3))[0]) / (2 * t)
    assert np.max(np.abs(H @ v - fd)) <= 1e-6 * np.abs(H @ v).max()
    assert abs(H - H.T).max() <= 1e-12 * abs(H).max()


def test_lumped_mass_totals_body_mass():
    X, tets = kuhn_grid(3, 4, 5, size=(0.3, 0.4, 0.5))
    mesh = Mesh.build(X, tets, 1e5, 0.45)
    m = lumped_mass(mesh, 1000.0)
    assert abs(m.sum() - 1000.0 * 0.3 * 0.4 * 0.5) <= 1e-12 * m.sum()


def test_energy_difference_matches_total_potential():
    rng = np.random.default_rng(10)
    sc = cube_compress(n=3, n_steps=4, ramp_steps=4)
    s = _stepper(sc)
    x = s.x + 0.01 * rng.standard_normal(s.x.shape)
    dx = 0.01 * rng.standard_normal(s.x.shape)
    for gam in (1.0, 0.5, 0.125):
        a = s.energy_difference(x, dx, gam)
        b = _total_potential(s, x + gam * dx) - _total_potential(s, x)
        assert abs(a - b) <= 1e-9 * max(abs(b), 1e-12) + 1e-10 * _total_potential(s, x)


# ---------------------------------------------------------------- P10: tiny meshes, dense checks
def _tiny_scenes():
    return [cube_compress(n=1, n_steps=4, ramp_steps=4), cube_compress(n=2, n_steps=4, ramp_steps=4),
            beam_twist(nx=4, ny=1, nz=1, L=0.2, W=0.05, n_steps=4, turns=0.5)]


@pytest.mark.parametrize("k", range(3))
def test_P10_pcg_and_descent_on_tiny_meshes(k):
    sc = _tiny_scenes()[k]
    s = _stepper(sc)
    rng = np.random.default_rng(11 + k)
    for trial in range(4):
        x = s.x.copy()
        x[:, 2] *= 1.0 - 0.2 * trial
        x += 0.01 * rng.standard_normal(x.shape)
        g, _, He, H = s.evaluate(x)
        Hd = H.toarray()
        # PN's matrix: every element projected, is SPD (dense Cholesky succeeds).
        Hp = s.asm.hessian(project_to_pd(He, 1e-8), s._diag()).toarray()
        np.linalg.cholesky(Hp)
        for M in (Hd, Hp):
            lmin = np.linalg.eigvalsh(M)[0]
            dx, ind, it = pcg_block_jacobi(__import__("scipy").sparse.csr_matrix(M), -g,
                                           diagonal_blocks(__import__("scipy").sparse.csr_matrix(M)))
            if lmin > 0:
                assert not ind
                assert np.linalg.norm(M @ dx + g) <= 1e-4 * np.linalg.norm(g) * (1 + 1e-9)
                xd = np.linalg.solve(M, -g)
                # |dx - x*| <= |r| / lambda_min for SPD M
                assert np.linalg.norm(dx - xd) <= np.linalg.norm(M @ dx + g) / lmin * (1 + 1e-6)
            if not ind:
                assert g @ dx < 0  # descent (Sec. 3, Eq. (3); Sec. 4.1 Newton-CG argument)


def test_pcg_detects_negative_curvature():
    import scipy.sparse as sps
    n = 9
    D = np.diag([4.0, 3.0, 2.0, 5.0, -1.0, 6.0, 1.0, 2.0, 3.0])
    M = sps.csr_matrix(D)
    blocks = np.stack([D[3 * i:3 * i + 3, 3 * i:3 * i + 3] for i in range(3)])
    _, ind, it = pcg_block_jacobi(M, np.ones(n), blocks)
    assert ind and it == 0  # diagonal block fails Sylvester
    # Indefinite matrix with SPD diagonal blocks: strong negative coupling between two vertices.
    A = np.eye(6) * 1.0
    A[0, 3] = A[3, 0] = 3.0
    M = sps.csr_matrix(A)
    blocks = np.stack([A[:3, :3], A[3:, 3:]])
    _, ind, it = pcg_block_jacobi(M, np.array([1.0, 0, 0, -1.0, 0, 0]), blocks)
    assert ind


# ---------------------------------------------------------------- P11: free fall is one exact Newton step
def test_P11_free_fall_exact():
    X, tets = kuhn_grid(2, 2, 2)
    sc = cube_compress(n=2, n_steps=2)
    p = Params(stop_mode="vel", stop_tol=1e-3)
    s = Stepper(X, tets, 0.0, 0.3, 1000.0, 1 / 30, (0, 0, -9.81), np.zeros(0, np.int32), p,
                x0=X, v0=np.tile([0.1, 0.0, 0.2], (X.shape[0], 1)))
    x0 = s.x.copy(); v0 = s.v.copy()
    st = s.step("PPN")
    h = 1 / 30
    expect = x0 + h * v0 + h * h * np.array([0, 0, -9.81])
    assert st.converged and st.newton_iters == 2 and st.projected == 0
    assert np.max(np.abs(s.x - expect)) <= 1e-14 * np.max(np.abs(expect))


# ---------------------------------------------------------------- P12: mode independence
def test_P12_modes_converge_to_same_positions():
    sc = cube_compress(n=4, n_steps=3, ramp_steps=6)
    xs = {}
    for mode in ("PN", "PDN", "PPN"):
        stp, stats = run_scene(sc, mode)
        assert all(s.converged for s in stats)
        xs[mode] = stp.x
    tol = 10 * sc.dt * sc.stop_tol
    assert np.max(np.abs(xs["PN"] - xs["PPN"])) <= tol
    assert np.max(np.abs(xs["PDN"] - xs["PPN"])) <= tol


# ---------------------------------------------------------------- P13: Algorithm 1 invariants
def test_P13_ppn_equals_newton_without_indefiniteness():
    sc = config(0, n_steps=3)
    a, sa = run_scene(sc, "PPN")
    b, sb = run_scene(sc, "PDN")
    assert all(s.projected == 0 and s.indefinite_solves == 0 for s in sa)
    assert np.array_equal(a.x, b.x)  # bit-identical: no projection ever happened

    # Pure Newton from the same start, written independently of the PPN control flow.
    s = _stepper(sc)
    s.x = sc.x0.copy()
    s.xhat = sc.x0 + sc.dt * sc.v0 + sc.dt ** 2 * np.asarray(sc.gravity)[None]
    x = s.x.copy()
    for k in range(100):
        g, _, _, H = s.evaluate(x)
        dx, ind, _ = pcg_block_jacobi(H, -g, diagonal_blocks(H))
        assert not ind
        dx = dx.reshape(-1, 3)
        if np.abs(dx).max() / sc.dt < sc.stop_tol:
            break
        gam = 1.0
        psi_x = element_psi(s.mesh, x)
        while s.energy_difference(x, dx, gam, psi_x) > 1e-4 * gam * (g @ dx.reshape(-1)):
            gam *= 0.5
        x = x + gam * dx
    c, _ = run_scene(sc, "PPN", n_steps=1)
    assert np.array_equal(c.x, x)


def test_P13_tiny_alpha_falls_back_to_PN_and_delta_is_power_of_two():
    sc = cube_compress(n=4, n_steps=2, ramp_steps=2)
    stp, st = run_scene(sc, "PPN", n_steps=1, trace=True, params=Params(alpha=1e-20, stop_mode="vel"))
    first = [r for r in st[0].trace if r["rounds"]]
    assert first, "scene must trigger indefiniteness"
    r0 = first[0]
    assert r0["rounds"][0][1] == sc.n_tets  # delta <= eps_delta: everything projected at once

    # With the default alpha, every delta is alpha^a beta^b |g|_inf exactly (powers of two).
    stp, st = run_scene(sc, "PPN", n_steps=2, trace=True)
    seen = 0
    for s in st:
        base = None
        for r in s.trace:
            for (delta, n_new, ind, it) in r["rounds"]:
                if base is None:
                    base = r["g_inf"] * 0.5
                ratio = delta / base
                m, e = math.frexp(ratio)
                assert m == 0.5, (delta, base)
                seen += 1
    assert seen > 0


def test_ppn_projects_fewer_than_pdn_on_compression():
    sc = cube_compress(n=6, n_steps=8, ramp_steps=8)
    res = {}
    for mode in ("PDN", "PPN"):
        _, st = run_scene(sc, mode)
        res[mode] = sum(s.projected for s in st)
    assert res["PPN"] < res["PDN"]


# ---------------------------------------------------------------- P14: numbering invariance
@pytest.mark.parametrize("mode", ["PN", "PDN", "PPN"])
def test_P14_results_do_not_depend_on_the_numbering(mode):
    """The method acts on the mesh, not on how its vertices and elements are
    numbered: a randomly renumbered scene (vertices, element order and each
    element's local order, orientation kept) takes the same Newton iterations
    and projects the same elements, and its positions mapped back agree up to
    the rounding of reordered sums.  An indexing slip (a transposed block, a
    local vertex taken in the wrong order, a scatter through the wrong map)
    breaks this on some numbering."""
    from scenes import renumbered
    sc = cube_compress(n=4, n_steps=4, ramp_steps=4)
    rn = renumbered(sc, seed=7)
    old, tmap = rn.meta["vertex_of_new"], rn.meta["tet_of_new"]
    runs = {}
    for s in (sc, rn):
        xs = []
        _, st = run_scene(s, mode, trace=True, callback=lambda n, S, _: xs.append(S.x.copy()))
        runs[s.name] = (xs, st)
    (xa, sa), (xb, sb) = runs[sc.name], runs[rn.name]
    assert sum(s.projected for s in sa) > 0 or mode == "PN"
    for a, b, ta, tb in zip(xa, xb, sa, sb):
        assert (ta.newton_iters, ta.projected, ta.inner_rounds) == (tb.newton_iters, tb.projected, tb.inner_rounds)
        assert np.max(np.abs(b - a[old])) <= 1e-12
        for ra, rb in zip(ta.trace, tb.trace):
            pa = ra.get("projected_idx", np.zeros(0, np.int32))
            pb = rb.get("projected_idx", np.zeros(0, np.int32))
            assert np.array_equal(np.sort(tmap[pb]), pa)
