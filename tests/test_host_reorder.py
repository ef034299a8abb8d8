"""The locality orderings (ppn_locality_order, host-only: it touches no
device) against what each order has to satisfy, without a GPU:

* both outputs are permutations, for both kinds;
* each order is a function of the geometry alone: a randomly renumbered copy
  of the same mesh gets the same sequence of physical vertices and elements;
* the pencil order of a regular grid is its lexicographic numbering with the
  shortest axis fastest and the longest slowest (the generator's own
  numbering when its axes are in that order);
* the Morton order of a 2^k grid with unit spacing ranks vertex (i, j, k) by
  the bit interleaving of i, j and k, written here bit by bit;
* elements follow their vertices (sorted by their new vertex ids);
* locality: on a randomly renumbered cube the mean index distance between
  the vertices of an element drops from about N/3 to that of the grid;
* errors: an empty mesh, an unknown kind, a vertex index out of range, a
  non-finite position.
"""
import numpy as np
import pytest

from paper_2505_21013_amd import PPNError, _abi, ppn_locality_order
from scenes import beam_twist, cube_compress, kuhn_grid, permuted, renumbered

KINDS = ["pencil", "morton"]


def _edge_span(tets):
    pairs = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    return float(np.concatenate([np.abs(tets[:, a].astype(np.int64) - tets[:, b]) for a, b in pairs]).mean())


@pytest.mark.parametrize("kind", KINDS)
def test_outputs_are_permutations_and_depend_on_geometry_only(kind):
    sc = cube_compress(n=8, n_steps=2, ramp_steps=2)
    rn = renumbered(sc, seed=3)
    vo, to = ppn_locality_order(sc.X, sc.tets, kind)
    vr, tr = ppn_locality_order(rn.X, rn.tets, kind)
    for p, n in ((vo, sc.n_verts), (to, sc.n_tets), (vr, sc.n_verts), (tr, sc.n_tets)):
        assert np.array_equal(np.sort(p), np.arange(n))
    assert np.array_equal(rn.meta["vertex_of_new"][vr], vo)
    assert np.array_equal(rn.meta["tet_of_new"][tr], to)


def test_pencil_order_of_a_grid_is_lexicographic():
    sc = beam_twist(nx=12, ny=3, nz=5, n_steps=2)       # extents 1.0 (x) > 0.2 (y) = 0.2 (z)
    rn = renumbered(sc, seed=1)
    vo, _ = ppn_locality_order(rn.X, rn.tets, "pencil")
    # the generator numbers (i, j, k) with k fastest: x slowest, then y, then z
    assert np.array_equal(rn.meta["vertex_of_new"][vo], np.arange(sc.n_verts))
    # a grid whose longest axis is z and shortest x: z slowest, x fastest
    X, tets = kuhn_grid(2, 3, 4, size=(0.2, 0.3, 0.4))
    vo, _ = ppn_locality_order(X, tets, "pencil")
    n = np.rint(X[vo] / 0.1).astype(np.int64)
    assert np.array_equal(np.lexsort((n[:, 0], n[:, 1], n[:, 2])), np.arange(len(vo)))


def test_morton_rank_is_the_bit_interleaving_on_a_power_of_two_grid():
    X, tets = kuhn_grid(7, 7, 7, size=(7.0, 7.0, 7.0))  # coordinates 0..7 on each axis
    vo, _ = ppn_locality_order(X, tets, "morton")
    ijk = np.rint(X[vo]).astype(np.int64)

    def interleave(i, j, k):
        key = 0
        for bit in range(3):
            key |= ((i >> bit) & 1) << (3 * bit)
            key |= ((j >> bit) & 1) << (3 * bit + 1)
            key |= ((k >> bit) & 1) << (3 * bit + 2)
        return key
    assert [interleave(*map(int, p)) for p in ijk] == list(range(len(ijk)))


@pytest.mark.parametrize("kind", KINDS)
def test_elements_follow_their_vertices_and_locality_is_restored(kind):
    base = cube_compress(n=16, n_steps=2, ramp_steps=2)
    sc = renumbered(base, seed=5)
    vo, to = ppn_locality_order(sc.X, sc.tets, kind)
    ordered = permuted(sc, vo, to)
    keys = np.sort(ordered.tets, axis=1)
    assert all(tuple(a) < tuple(b) for a, b in zip(keys[:-1], keys[1:]))
    assert _edge_span(sc.tets) > 0.25 * sc.n_verts
    assert _edge_span(ordered.tets) < 1.5 * _edge_span(base.tets)


def test_errors():
    X, tets = kuhn_grid(1, 1, 1)
    with pytest.raises(PPNError, match="outside"):
        ppn_locality_order(X, np.where(tets == 3, 99, tets))
    bad = X.copy()
    bad[2, 1] = np.nan
    with pytest.raises(PPNError, match="not finite"):
        ppn_locality_order(bad, tets, "morton")
    with pytest.raises(PPNError, match="empty"):
        ppn_locality_order(X, np.zeros((0, 4), np.int32))
    vo = np.empty(len(X), np.int32)
    to = np.empty(len(tets), np.int32)
    code = _abi.lib().ppn_locality_order(len(X), X.ctypes.data_as(_abi.dp), len(tets),
                                         np.ascontiguousarray(tets, np.int32).ctypes.data_as(_abi.ip), 7,
                                         vo.ctypes.data_as(_abi.ip), to.ctypes.data_as(_abi.ip))
    assert code != 0 and b"unknown ordering kind 7" in _abi.lib().ppn_last_error(None)
    code = _abi.lib().ppn_locality_order(len(X), None, len(tets), None, 0, None, None)
    assert code != 0 and b"rest_xyz must not be NULL" in _abi.lib().ppn_last_error(None)
