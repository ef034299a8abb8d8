"""The seeded scene generator: sizes, orientation, determinism and Dirichlet sets."""
import numpy as np
import pytest

from scenes import config, kuhn_grid


def _edges(tets, n):
    pairs = np.concatenate([np.sort(tets[:, [a, b]], axis=1) for a in range(4) for b in range(a + 1, 4)])
    return np.unique(pairs[:, 0].astype(np.int64) * n + pairs[:, 1]).size


@pytest.mark.parametrize("k,nv,nt,ne", [(0, 343, 1296, 1854), (1, 23409, 122880, 151920)])
def test_sizes(k, nv, nt, ne):
    s = config(k)
    assert s.n_verts == nv and s.n_tets == nt and _edges(s.tets, nv) == ne


def test_cube64_sizes_and_log_uniform_E():
    s = config(2)
    assert (s.n_verts, s.n_tets) == (274625, 1572864)
    assert s.E.min() >= 1e4 and s.E.max() <= 1e6
    lg = np.log10(s.E)
    assert abs(lg.mean() - 5.0) < 0.01 and abs(np.median(lg) - 5.0) < 0.01


def test_positive_orientation_and_conforming():
    X, tets = kuhn_grid(3, 2, 4, size=(0.3, 0.2, 0.4))
    D = np.stack([X[tets[:, a]] - X[tets[:, 0]] for a in (1, 2, 3)], axis=-1)
    vol = np.linalg.det(D) / 6
    assert np.all(vol > 0) and abs(vol.sum() - 0.3 * 0.2 * 0.4) < 1e-14
    # conforming: every interior face is shared by exactly two tets, boundary faces by one
    faces = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]]), axis=1)
    _, cnt = np.unique(faces, axis=0, return_counts=True)
    assert set(np.unique(cnt)) <= {1, 2}
    assert (cnt == 1).sum() == 2 * 2 * (3 * 2 + 2 * 4 + 3 * 4)


def test_seeded_and_schedules():
    a, b = config(0), config(0)
    assert np.array_equal(a.x0, b.x0)
    cell = 1.0 / 6
    assert np.abs(a.x0 - a.X).max() <= 0.05 * cell and np.abs(a.x0 - a.X).max() > 0.04 * cell
    assert np.array_equal(a.targets(5), a.X[a.dirichlet_ids])
    s = config(1)
    t0 = s.targets(0)
    t25 = s.targets(25)  # 2 turns over 100 steps: half a turn at step 25
    right = s.X[s.dirichlet_ids, 0] == 1.0
    assert np.allclose(t0, s.X[s.dirichlet_ids])
    r0 = t0[right, 1:] - 0.1
    r1 = t25[right, 1:] - 0.1
    assert np.allclose(r1, -r0)


def test_renumbered_is_the_same_mesh():
    """A renumbered scene holds the same elements (as vertex sets mapped back),
    keeps every orientation, and carries materials, states and the boundary
    schedule along with the new numbering."""
    from scenes import cube_compress, renumbered
    s = cube_compress(n=4, n_steps=6, ramp_steps=6)
    r = renumbered(s, seed=7)
    old, tmap = r.meta["vertex_of_new"], r.meta["tet_of_new"]
    assert sorted(old.tolist()) == list(range(s.n_verts)) and sorted(tmap.tolist()) == list(range(s.n_tets))
    assert not np.array_equal(old, np.arange(s.n_verts))
    assert np.array_equal(np.sort(old[r.tets], axis=1), np.sort(s.tets[tmap], axis=1))
    assert not np.array_equal(old[r.tets], s.tets[tmap])          # local orders changed too
    D = np.stack([r.X[r.tets[:, a]] - r.X[r.tets[:, 0]] for a in (1, 2, 3)], axis=-1)
    D0 = np.stack([s.X[s.tets[tmap, a]] - s.X[s.tets[tmap, 0]] for a in (1, 2, 3)], axis=-1)
    assert np.allclose(np.linalg.det(D), np.linalg.det(D0), rtol=1e-12, atol=0)
    assert np.array_equal(r.X, s.X[old]) and np.array_equal(r.x0, s.x0[old])
    assert np.array_equal(r.E, s.E[tmap]) and np.array_equal(r.nu, s.nu[tmap])
    assert np.all(np.diff(r.dirichlet_ids) > 0)
    for n in (0, 3, 6):
        got = dict(zip(old[r.dirichlet_ids].tolist(), map(tuple, r.targets(n))))
        want = dict(zip(s.dirichlet_ids.tolist(), map(tuple, s.targets(n))))
        assert got == want


def test_renumbering_twice_composes_the_maps():
    """A renumbered copy of a renumbered scene keeps maps to the original ids."""
    from scenes import cube_compress, renumbered
    s = cube_compress(n=3, n_steps=2, ramp_steps=2)
    r2 = renumbered(renumbered(s, seed=1), seed=2)
    old, tmap = r2.meta["vertex_of_new"], r2.meta["tet_of_new"]
    assert np.array_equal(r2.X, s.X[old]) and np.array_equal(r2.E, s.E[tmap])
    assert np.array_equal(np.sort(old[r2.tets], axis=1), np.sort(s.tets[tmap], axis=1))
