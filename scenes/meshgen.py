"""Seeded synthetic scenes: tetrahedral meshes, materials and Dirichlet schedules.

This module only generates inputs.  It holds none of the method's arithmetic
(no energies, derivatives, projections or solves), so both the CPU oracle and
the GPU library take their scenes from here.

Meshes are regular grids of hexahedral cells, each split into six tetrahedra
along the cell diagonal (0,0,0)->(1,1,1) (the Kuhn / Freudenthal split).  The
six tetrahedra of a cell are the six monotone lattice paths from the cell's
low corner to its high corner, one per permutation of the three axes.  For an
odd permutation the second and third vertices are swapped, which makes every
tetrahedron positively oriented; the orientation follows from the parity of
the permutation alone, so no determinant is evaluated here.

Parameter ranges follow the paper's scene table (Sec. 5.1, Table 1):
Young's modulus 1e4..1e6 Pa, Poisson ratio 0.40..0.49, density 1000 kg/m^3,
time steps 1/30 and 1/60 s.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)

# Permutations of the axes in lexicographic order, with their parity.
_PERMS = list(itertools.permutations((0, 1, 2)))
_ODD = {(0, 2, 1), (1, 0, 2), (2, 1, 0)}


def kuhn_grid(nx: int, ny: int, nz: int, size=(1.0, 1.0, 1.0)):
    """Vertices (N,3) float64 and tetrahedra (T,4) int32 of an nx*ny*nz grid.

    Vertex id = (i*(ny+1) + j)*(nz+1) + k; cells in lexicographic (i, j, k)
    order; six tetrahedra per cell in permutation order.
    """
    nvx, nvy, nvz = nx + 1, ny + 1, nz + 1
    ii, jj, kk = np.meshgrid(np.arange(nvx), np.arange(nvy), np.arange(nvz), indexing="ij")
    X = np.stack([ii.ravel() * (size[0] / nx),
                  jj.ravel() * (size[1] / ny),
                  kk.ravel() * (size[2] / nz)], axis=1).astype(np.float64)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()

    def vid(di, dj, dk):
        return ((ci + di) * nvy + (cj + dj)) * nvz + (ck + dk)

    tets = np.empty((ci.size, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        off = [0, 0, 0]
        path = [vid(*off)]
        for ax in perm:
            off[ax] += 1
            path.append(vid(*off))
        if perm in _ODD:
            path[1], path[2] = path[2], path[1]
        tets[:, p, :] = np.stack(path, axis=1)
    return X, tets.reshape(-1, 4).astype(np.int32)


@dataclass
class Scene:
    """Everything one simulation run needs, independent of the solver."""
    name: str
    X: np.ndarray                 # rest positions (N,3) [m]
    tets: np.ndarray              # (T,4) int32
    x0: np.ndarray                # initial positions (N,3)
    v0: np.ndarray                # initial velocities (N,3)
    E: np.ndarray                 # Young's modulus per element (T,) [Pa]
    nu: np.ndarray                # Poisson ratio per element (T,)
    rho: float                    # density [kg/m^3]
    dt: float                     # time step [s]
    gravity: tuple
    dirichlet_ids: np.ndarray     # (n_D,) int32, ascending
    targets: Callable[[int], np.ndarray] = field(repr=False)  # step n -> (n_D,3) targets at t_n
    n_steps: int = 1
    stop_mode: str = "vel"        # "vel": dt^-1 |dx|_inf < tol ; "grad_rel": |g|_2 <= tol |g0|_2
    stop_tol: float = 1e-3
    meta: dict = field(default_factory=dict)

    @property
    def n_verts(self) -> int:
        return self.X.shape[0]

    @property
    def n_tets(self) -> int:
        return self.tets.shape[0]


def _face(X, axis, value, atol=1e-12):
    return np.nonzero(np.abs(X[:, axis] - value) <= atol)[0].astype(np.int32)


def cube_jitter(n=6, E=1e5, nu=0.45, rho=1000.0, dt=1.0 / 60.0, jitter=0.05, seed=0,
                n_steps=20, newton_rel_tol=1e-6) -> Scene:
    """Small parity scene: unit cube of n^3 cells, bottom face pinned to rest,
    gravity, every initial vertex jittered by U(-jitter*cell, +jitter*cell).

    Newton stops once the step is below ``newton_rel_tol`` of the body's size
    (the rest bounding-box diagonal), expressed as the velocity criterion
    |dx|_inf / dt < newton_rel_tol * diag / dt."""
    X, tets = kuhn_grid(n, n, n)
    cell = 1.0 / n
    rng = np.random.default_rng(seed)
    x0 = X + rng.uniform(-jitter * cell, jitter * cell, size=X.shape)
    ids = _face(X, 2, 0.0)
    tgt = X[ids].copy()
    T = tets.shape[0]
    return Scene(name=f"cube{n}_jitter", X=X, tets=tets, x0=x0, v0=np.zeros_like(X),
                 E=np.full(T, E), nu=np.full(T, nu), rho=rho, dt=dt, gravity=GRAVITY,
                 dirichlet_ids=ids, targets=lambda step: tgt, n_steps=n_steps,
                 stop_mode="vel", stop_tol=newton_rel_tol * math.sqrt(3.0) / dt,
                 meta=dict(cells=(n, n, n), size=(1.0, 1.0, 1.0), newton_rel_tol=newton_rel_tol))


def beam_twist(nx=80, ny=16, nz=16, L=1.0, W=0.2, E=1e5, nu=0.45, rho=1000.0, dt=1.0 / 30.0,
               turns=2.0, n_steps=100) -> Scene:
    """Beam fixed at x = 0; the x = L face is driven to c + R_x(theta_n)(X - c)
    with theta_n = 2*pi*turns*n/n_steps (c = face centre)."""
    X, tets = kuhn_grid(nx, ny, nz, size=(L, W, W))
    left = _face(X, 0, 0.0)
    right = _face(X, 0, L)
    ids = np.concatenate([left, right]).astype(np.int32)
    order = np.argsort(ids, kind="stable")
    ids = ids[order]
    base = X[ids].copy()
    is_right = np.isin(ids, right)
    c = np.array([L, W / 2, W / 2])

    def targets(step):
        th = 2.0 * math.pi * turns * step / n_steps
        ct, st = math.cos(th), math.sin(th)
        t = base.copy()
        r = base[is_right] - c
        t[is_right, 1] = c[1] + ct * r[:, 1] - st * r[:, 2]
        t[is_right, 2] = c[2] + st * r[:, 1] + ct * r[:, 2]
        return t

    T = tets.shape[0]
    return Scene(name=f"beam{nx}x{ny}x{nz}_twist", X=X, tets=tets, x0=X.copy(),
                 v0=np.zeros_like(X), E=np.full(T, E), nu=np.full(T, nu), rho=rho, dt=dt,
                 gravity=GRAVITY, dirichlet_ids=ids, targets=targets, n_steps=n_steps,
                 stop_mode="vel", stop_tol=1e-3,
                 meta=dict(cells=(nx, ny, nz), size=(L, W, W)))


def cube_compress(n=64, L=1.0, E_lo=1e4, E_hi=1e6, nu=0.48, rho=1000.0, dt=1.0 / 30.0,
                  squash=0.6, ramp_steps=50, n_steps=50, seed=2) -> Scene:
    """Cube pinned at z = 0; the top face is driven to (X, Y, L(1 - squash*min(1, n/ramp)))
    while E is drawn log-uniformly per element."""
    X, tets = kuhn_grid(n, n, n, size=(L, L, L))
    rng = np.random.default_rng(seed)
    T = tets.shape[0]
    E = np.exp(rng.uniform(math.log(E_lo), math.log(E_hi), size=T))
    bot = _face(X, 2, 0.0)
    top = _face(X, 2, L)
    ids = np.sort(np.concatenate([bot, top])).astype(np.int32)
    base = X[ids].copy()
    is_top = np.isin(ids, top)

    def targets(step):
        t = base.copy()
        t[is_top, 2] = L * (1.0 - squash * min(1.0, step / ramp_steps))
        return t

    return Scene(name=f"cube{n}_compress", X=X, tets=tets, x0=X.copy(), v0=np.zeros_like(X),
                 E=E, nu=np.full(T, nu), rho=rho, dt=dt, gravity=GRAVITY,
                 dirichlet_ids=ids, targets=targets, n_steps=n_steps,
                 stop_mode="vel", stop_tol=1e-3,
                 meta=dict(cells=(n, n, n), size=(L, L, L)))


def block_rotate(nx, ny, nz, cell, axis, angle, E=1e5, nu=0.45, rho=1000.0, dt=1.0 / 30.0,
                 ramp_steps=20, name="block") -> Scene:
    """Block of nx*ny*nz cells of edge ``cell``; the x = 0 face is pinned and
    the opposite face is driven to c + R(axis, theta_n)(X - c), c its centre,
    theta_n = angle * min(1, n / ramp_steps) (Rodrigues' rotation about the
    unit ``axis``)."""
    size = (nx * cell, ny * cell, nz * cell)
    X, tets = kuhn_grid(nx, ny, nz, size=size)
    left = _face(X, 0, 0.0)
    right = _face(X, 0, size[0], atol=1e-9 * size[0])
    ids = np.sort(np.concatenate([left, right])).astype(np.int32)
    base = X[ids].copy()
    is_right = np.isin(ids, right)
    c = np.array([size[0], size[1] / 2, size[2] / 2])
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)

    def targets(step):
        th = angle * min(1.0, step / ramp_steps)
        r = base[is_right] - c
        ct, st = math.cos(th), math.sin(th)
        rot = r * ct + np.cross(a, r) * st + np.outer(r @ a, a) * (1.0 - ct)
        t = base.copy()
        t[is_right] = c + rot
        return t

    T = tets.shape[0]
    return Scene(name=name, X=X, tets=tets, x0=X.copy(), v0=np.zeros_like(X),
                 E=np.full(T, E), nu=np.full(T, nu), rho=rho, dt=dt, gravity=GRAVITY,
                 dirichlet_ids=ids, targets=targets, n_steps=ramp_steps, stop_mode="vel",
                 stop_tol=1e-3, meta=dict(cells=(nx, ny, nz), size=size, axis=tuple(a),
                                          angle=angle))


def batch_scenes(n_scenes=64, seed=3, n_lo=4, n_hi=40, ramp_steps=20):
    """Independent scenes for batched stepping: n = round(n_lo (n_hi/n_lo)^U)
    cells per side, a cube n^3 or a beam n x ceil(n/4) x ceil(n/4) (coin flip)
    with cells of 1/n m, E 1e5 Pa, nu 0.45, rho 1000, h 1/30; the x = 0 face
    pinned and the far face rotated about a random unit axis through its
    centre by a total angle U(0, pi) over ``ramp_steps`` steps."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        n = int(round(n_lo * (n_hi / n_lo) ** rng.uniform()))
        beam = bool(rng.integers(2))
        axis = rng.standard_normal(3)
        angle = float(rng.uniform(0.0, math.pi))
        dims = (n, -(-n // 4), -(-n // 4)) if beam else (n, n, n)
        out.append(block_rotate(*dims, cell=1.0 / n, axis=axis, angle=angle, ramp_steps=ramp_steps,
                                name=f"s{k}_{'beam' if beam else 'cube'}{n}"))
    return out


def serving_scenes(n_scenes=128, seed=4, t_lo=1e3, t_hi=5e5, ramp_steps=20):
    """Resident scenes for the serving loop: target tet counts log-uniform in
    [t_lo, t_hi], cubes of n = round((T/6)^(1/3)) cells of 1/n m, material and
    constraints as in batch_scenes."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        T = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
        n = max(1, int(round((T / 6.0) ** (1.0 / 3.0))))
        axis = rng.standard_normal(3)
        angle = float(rng.uniform(0.0, math.pi))
        out.append(block_rotate(n, n, n, cell=1.0 / n, axis=axis, angle=angle, ramp_steps=ramp_steps,
                                name=f"r{k}_cube{n}"))
    return out


# The twelve even permutations of a tetrahedron's four local vertices: each
# keeps the orientation (the sign of the volume) of the element it reorders.
_EVEN4 = [q for q in itertools.permutations(range(4))
          if sum(q[i] > q[j] for i in range(4) for j in range(i + 1, 4)) % 2 == 0]


def permuted(sc: Scene, vertex_order, tet_order, local=None, name=None) -> Scene:
    """The same scene numbered anew: new vertex v is old vertex_order[v], new
    element e is old element tet_order[e], and (if given) local[e] reorders
    the new element's four vertices.  Geometry, materials and the boundary
    schedule are carried along; the Dirichlet ids stay ascending, their
    targets reordered with them.  The maps are kept in ``meta["vertex_of_new"]``
    and ``meta["tet_of_new"]`` (composed with any the scene already had)."""
    old_of_new = np.asarray(vertex_order, np.int64)
    tet_of_new = np.asarray(tet_order, np.int64)
    nv, nt = sc.n_verts, sc.n_tets
    assert np.array_equal(np.sort(old_of_new), np.arange(nv)), "vertex_order is not a permutation"
    assert np.array_equal(np.sort(tet_of_new), np.arange(nt)), "tet_order is not a permutation"
    new_of_old = np.empty(nv, np.int64)
    new_of_old[old_of_new] = np.arange(nv)
    tets = new_of_old[sc.tets[tet_of_new]]
    if local is not None:
        tets = np.take_along_axis(tets, np.asarray(local, np.int64), axis=1)
    ids = new_of_old[sc.dirichlet_ids]
    order = np.argsort(ids, kind="stable")
    src_targets = sc.targets
    meta = dict(sc.meta)
    meta["vertex_of_new"] = np.asarray(sc.meta.get("vertex_of_new", np.arange(nv)))[old_of_new]
    meta["tet_of_new"] = np.asarray(sc.meta.get("tet_of_new", np.arange(nt)))[tet_of_new]
    return Scene(name=name or f"{sc.name}_perm", X=sc.X[old_of_new].copy(), tets=tets.astype(np.int32),
                 x0=sc.x0[old_of_new].copy(), v0=sc.v0[old_of_new].copy(),
                 E=sc.E[tet_of_new].copy(), nu=sc.nu[tet_of_new].copy(), rho=sc.rho, dt=sc.dt,
                 gravity=sc.gravity, dirichlet_ids=ids[order].astype(np.int32),
                 targets=lambda step: np.asarray(src_targets(step))[order],
                 n_steps=sc.n_steps, stop_mode=sc.stop_mode, stop_tol=sc.stop_tol, meta=meta)


def renumbered(sc: Scene, seed: int = 0) -> Scene:
    """The same scene with its vertices and elements numbered at random:
    vertex ids permuted, the element list shuffled, and each element's local
    vertices reordered by a random even permutation (which keeps its
    orientation)."""
    rng = np.random.default_rng(seed)
    vo = rng.permutation(sc.n_verts)
    to = rng.permutation(sc.n_tets)
    local = np.array(_EVEN4, np.int64)[rng.integers(0, len(_EVEN4), sc.n_tets)]
    return permuted(sc, vo, to, local, name=f"{sc.name}_renum{seed}")


def config(k: int, **kw):
    """The workload configurations by index: 0 small parity cube, 1 twisted
    beam (122,880 tets), 2 compressed heterogeneous cube (1,572,864 tets),
    3 a batch of 64 independent scenes (a list), 4 the 128 resident scenes of
    the serving loop (a list)."""
    if k == 0:
        return cube_jitter(**kw)
    if k == 1:
        return beam_twist(**kw)
    if k == 2:
        return cube_compress(**kw)
    if k == 3:
        return batch_scenes(**kw)
    if k == 4:
        return serving_scenes(**kw)
    raise ValueError(f"unknown configuration {k}")
