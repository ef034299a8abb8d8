"""MI355X (gfx950) implementation of Progressively Projected Newton (arXiv 2505.21013).

The hot path lives in ``libppn.so`` (hand-written HIP, see ``csrc/``) behind the
C ABI of ``include/ppn.h``.  This module only marshals arguments: functions
keep the C names (``ppn_newton_step`` ...) and ``Scene`` is a thin object
wrapper over one handle.  PyTorch may supply the HIP stream and destination
device buffers; nothing here computes any part of the method.
"""
import ctypes as C

import numpy as np

from . import _abi
from ._abi import (MODES, PPN_FP64, PPN_MIXED, PPN_NOALLOC_MAX_ELEMENTS, PPN_ORDER_MORTON,
                   PPN_ORDER_PENCIL, PPN_PDN, PPN_PN,
                   PPN_PPN, PPN_STOP_GRAD_REL, PPN_STOP_VEL, STATUS, ppn_engine_info, ppn_iter_record,
                   ppn_params, ppn_scene_desc, ppn_step_stats)

__all__ = ["Scene", "Engine", "PPNError", "ppn_params_default", "ppn_project_batch_dev", "ppn_locality_order",
           "ppn_params", "ppn_step_stats", "ppn_iter_record", "MODES", "PPN_PN", "PPN_PDN", "PPN_PPN",
           "PPN_FP64", "PPN_MIXED", "PPN_STOP_VEL", "PPN_STOP_GRAD_REL", "PPN_ORDER_PENCIL",
           "PPN_ORDER_MORTON", "library_path"]


class PPNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def library_path():
    return _abi.LIB_PATH


def _d(a):
    return a.ctypes.data_as(_abi.dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_abi.ip) if a is not None else None


def _u8(a):
    return a.ctypes.data_as(_abi.u8p) if a is not None else None


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _mask(m, T):
    if m is None:
        return None
    m = np.ascontiguousarray(m, dtype=np.uint8).reshape(-1)
    if m.size != T:
        raise ValueError("mask must have one entry per element")
    return m


def _check(code, handle=None, warn_ok=False):
    if code < 0 or (code > 0 and not warn_ok):
        msg = _abi.lib().ppn_last_error(handle)
        raise PPNError(code, msg.decode() if msg else "")
    return code


def ppn_params_default():
    p = ppn_params()
    _check(_abi.lib().ppn_params_default(C.byref(p)))
    return p


def ppn_project_batch_dev(H_dev, Hhat_dev, n, eps=1e-8, stream=None):
    """Project n row-major 12x12 matrices in device memory (pointers or torch tensors)."""
    def ptr(t):
        return C.c_void_p(t.data_ptr() if hasattr(t, "data_ptr") else int(t))
    _check(_abi.lib().ppn_project_batch_dev(ptr(H_dev), ptr(Hhat_dev), int(n), float(eps),
                                           C.c_void_p(stream) if stream else None))


def ppn_locality_order(rest_xyz, tets, kind="pencil"):
    """(vertex_order, tet_order), new -> old ids of a numbering with spatial
    locality; kind "pencil" (banded sweep) or "morton" (Z-order curve)."""
    kind = {"pencil": PPN_ORDER_PENCIL, "morton": PPN_ORDER_MORTON}[kind]
    X = _f64(rest_xyz).reshape(-1, 3)
    tt = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    vo = np.empty(X.shape[0], np.int32)
    to = np.empty(tt.shape[0], np.int32)
    _check(_abi.lib().ppn_locality_order(X.shape[0], _d(X), tt.shape[0], _i(tt), kind, _i(vo), _i(to)))
    return vo, to


class Scene:
    """One simulation scene on the current HIP device (see include/ppn.h)."""

    def __init__(self, stream=None, precision=PPN_FP64):
        self._h = C.c_void_p()
        _check(_abi.lib().ppn_scene_create(C.byref(self._h), C.c_void_p(stream) if stream else None,
                                          precision))
        self.N = 0
        self.T = 0

    def close(self):
        if self._h:
            _abi.lib().ppn_scene_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _c(self, code, warn_ok=False):
        return _check(code, self._h, warn_ok)

    # -- set-up ------------------------------------------------------------------
    def ppn_load_mesh(self, rest_xyz, tets, init_xyz=None):
        X = _f64(rest_xyz).reshape(-1, 3)
        tt = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        x0 = None if init_xyz is None else _f64(init_xyz, X.size)
        self._c(_abi.lib().ppn_load_mesh(self._h, X.shape[0], _d(X), tt.shape[0], _i(tt), _d(x0)))
        self.N, self.T = X.shape[0], tt.shape[0]

    def ppn_set_material(self, rho, E, nu):
        E = np.atleast_1d(_f64(E))
        nu = np.atleast_1d(_f64(nu))
        per = int(E.size > 1 or nu.size > 1)
        if per:
            E = np.broadcast_to(E, (self.T,)).copy()
            nu = np.broadcast_to(nu, (self.T,)).copy()
        self._c(_abi.lib().ppn_set_material(self._h, float(rho), _d(E), _d(nu), per))

    def ppn_set_time_step(self, dt, gravity=(0.0, 0.0, -9.81)):
        g = _f64(gravity, 3)
        self._c(_abi.lib().ppn_set_time_step(self._h, float(dt), _d(g)))

    def ppn_set_dirichlet(self, ids, targets):
        ids = np.ascontiguousarray(ids, dtype=np.int32).reshape(-1)
        t = _f64(targets, 3 * ids.size)
        self._c(_abi.lib().ppn_set_dirichlet(self._h, ids.size, _i(ids), _d(t)))

    def ppn_set_params(self, params=None, **kw):
        p = ppn_params_default() if params is None else params
        for k, v in kw.items():
            if k == "stop_mode" and isinstance(v, str):
                v = {"vel": PPN_STOP_VEL, "grad_rel": PPN_STOP_GRAD_REL}[v]
            setattr(p, k, v)
        self._c(_abi.lib().ppn_set_params(self._h, C.byref(p)))
        return p

    def ppn_set_profiling(self, enable=True):
        self._c(_abi.lib().ppn_set_profiling(self._h, int(bool(enable))))

    def ppn_set_trace(self, enable=True):
        self._c(_abi.lib().ppn_set_trace(self._h, int(bool(enable))))

    # -- stepping ----------------------------------------------------------------
    def ppn_newton_step(self, mode="PPN"):
        st = ppn_step_stats()
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        code = self._c(_abi.lib().ppn_newton_step(self._h, m, C.byref(st)), warn_ok=True)
        d = st.as_dict()
        d["status"] = STATUS.get(code, code)
        return d

    def ppn_get_positions(self):
        out = np.empty((self.N, 3))
        self._c(_abi.lib().ppn_get_positions(self._h, _d(out)))
        return out

    def ppn_get_positions_dev(self, tensor, stream=None):
        """Device-to-device copy into a float64 tensor of 3N elements on the scene's device."""
        if tensor.numel() != 3 * self.N or str(tensor.dtype) != "torch.float64" or not tensor.is_contiguous():
            raise ValueError("need a contiguous float64 tensor with 3*N elements")
        self._c(_abi.lib().ppn_get_positions_dev(self._h, C.c_void_p(tensor.data_ptr()),
                                                C.c_void_p(stream) if stream else None))

    def ppn_get_state(self):
        x = np.empty((self.N, 3))
        v = np.empty((self.N, 3))
        self._c(_abi.lib().ppn_get_state(self._h, _d(x), _d(v)))
        return x, v

    def ppn_set_state(self, x, v):
        x = _f64(x, 3 * self.N)
        v = _f64(v, 3 * self.N)
        self._c(_abi.lib().ppn_set_state(self._h, _d(x), _d(v)))

    def ppn_get_last_stats(self):
        st = ppn_step_stats()
        self._c(_abi.lib().ppn_get_last_stats(self._h, C.byref(st)))
        return st.as_dict()

    def ppn_scene_info(self):
        n, t, e = C.c_int32(), C.c_int32(), C.c_int32()
        nb, by = C.c_int64(), C.c_int64()
        self._c(_abi.lib().ppn_scene_info(self._h, C.byref(n), C.byref(t), C.byref(e), C.byref(nb),
                                         C.byref(by)))
        return dict(n_verts=n.value, n_tets=t.value, n_edges=e.value, n_blocks=nb.value,
                    device_bytes=by.value)

    def ppn_trace(self):
        """Records of the last step: list of dicts, each with 'projected_ids'."""
        cnt = C.c_int32()
        self._c(_abi.lib().ppn_trace_count(self._h, C.byref(cnt)))
        out = []
        for i in range(cnt.value):
            rec = ppn_iter_record()
            self._c(_abi.lib().ppn_trace_get(self._h, i, C.byref(rec), None))
            ids = np.empty(max(rec.n_projected, 1), dtype=np.int32)
            self._c(_abi.lib().ppn_trace_get(self._h, i, C.byref(rec), _i(ids)))
            d = rec.as_dict()
            d["projected_ids"] = ids[:rec.n_projected].copy()
            out.append(d)
        return out

    # -- single stages -----------------------------------------------------------
    def ppn_eval_gradient(self, x):
        x = _f64(x, 3 * self.N)
        g = np.empty(3 * self.N)
        self._c(_abi.lib().ppn_eval_gradient(self._h, _d(x), _d(g)))
        return g

    def ppn_eval_element_hessians(self, x, ids=None, proj_mask=None):
        x = _f64(x, 3 * self.N)
        ids_a = None if ids is None else np.ascontiguousarray(ids, dtype=np.int32).reshape(-1)
        n = self.T if ids_a is None else ids_a.size
        out = np.empty((n, 12, 12))
        m = _mask(proj_mask, self.T)
        self._c(_abi.lib().ppn_eval_element_hessians(self._h, _d(x), _u8(m), n, _i(ids_a), _d(out)))
        return out

    def ppn_eval_element_hessians_noalloc(self, x, ids=None, proj_mask=None):
        """As ppn_eval_element_hessians, staged in the library's fixed device
        array (no device allocation; at most PPN_NOALLOC_MAX_ELEMENTS matrices)."""
        x = _f64(x, 3 * self.N)
        ids_a = None if ids is None else np.ascontiguousarray(ids, dtype=np.int32).reshape(-1)
        n = self.T if ids_a is None else ids_a.size
        out = np.empty((n, 12, 12))
        m = _mask(proj_mask, self.T)
        self._c(_abi.lib().ppn_eval_element_hessians_noalloc(self._h, _d(x), _u8(m), n, _i(ids_a), _d(out)))
        return out

    def ppn_eval_hessian(self, x, proj_mask=None):
        """(row_ptr, col, vals[nb,3,3]) of the assembled block-sparse Hessian."""
        info = self.ppn_scene_info()
        x = _f64(x, 3 * self.N)
        rp = np.empty(self.N + 1, dtype=np.int32)
        col = np.empty(info["n_blocks"], dtype=np.int32)
        vals = np.empty((info["n_blocks"], 3, 3))
        m = _mask(proj_mask, self.T)
        self._c(_abi.lib().ppn_eval_hessian(self._h, _d(x), _u8(m), _i(rp), _i(col), _d(vals)))
        return rp, col, vals

    def ppn_select(self, g, delta, proj_in=None):
        g = _f64(g, 3 * self.N)
        m = _mask(proj_in, self.T)
        out = np.empty(self.T, dtype=np.uint8)
        cnt = C.c_int32()
        self._c(_abi.lib().ppn_select(self._h, _d(g), float(delta), _u8(m), _u8(out), C.byref(cnt)))
        return out, cnt.value

    def ppn_debug_iterate(self, x, delta_in=float("inf"), mode="PPN"):
        """(mask of projected elements, delta_out, ind) of one Newton iteration from x."""
        x = _f64(x, 3 * self.N)
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        mask = np.empty(self.T, np.uint8)
        dout, ind = C.c_double(), C.c_int32()
        self._c(_abi.lib().ppn_debug_iterate(self._h, m, _d(x), float(delta_in), _u8(mask), C.byref(dout),
                                            C.byref(ind)))
        return mask, dout.value, bool(ind.value)

    def ppn_solve(self, x, proj_mask=None):
        x = _f64(x, 3 * self.N)
        dx = np.empty(3 * self.N)
        ind, it = C.c_int32(), C.c_int32()
        m = _mask(proj_mask, self.T)
        self._c(_abi.lib().ppn_solve(self._h, _d(x), _u8(m), _d(dx), C.byref(ind), C.byref(it)))
        return dx, bool(ind.value), it.value

    def ppn_hessian_product(self, x, d, proj_mask=None):
        x = _f64(x, 3 * self.N)
        d = _f64(d, 3 * self.N)
        q = np.empty(3 * self.N)
        m = _mask(proj_mask, self.T)
        self._c(_abi.lib().ppn_hessian_product(self._h, _d(x), _u8(m), _d(d), _d(q)))
        return q

    def ppn_energy_difference(self, x, dx, gammas):
        x = _f64(x, 3 * self.N)
        dx = _f64(dx, 3 * self.N)
        g = _f64(gammas).reshape(-1)
        out = np.empty(g.size)
        self._c(_abi.lib().ppn_energy_difference(self._h, _d(x), _d(dx), g.size, _d(g), _d(out)))
        return out


class Engine:
    """Serving engine (``ppn_engine_*``): resident scenes stepped on request by
    ``n_workers`` host threads, one HIP stream per resident scene."""

    def __init__(self, n_workers=8, mem_budget_bytes=0):
        h = C.c_void_p()
        _check(_abi.lib().ppn_engine_create(C.byref(h), int(n_workers), int(mem_budget_bytes)))
        self._h = h
        self._keep = {}

    def close(self):
        if self._h:
            _abi.lib().ppn_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def ppn_engine_add_scene(self, X, tets, E, nu, rho, dt, gravity, dirichlet_ids, precision=PPN_FP64,
                             params=None, x0=None, v0=None):
        X = _f64(X)
        N = X.size // 3
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        E = _f64(E).reshape(-1)
        nu = _f64(nu).reshape(-1)
        ids = np.ascontiguousarray(dirichlet_ids, dtype=np.int32)
        d = ppn_scene_desc()
        d.n_verts, d.n_tets = N, tets.shape[0]
        d.rest_xyz, d.tets = _d(X), _i(tets)
        x0 = _f64(x0, 3 * N) if x0 is not None else None
        v0 = _f64(v0, 3 * N) if v0 is not None else None
        d.init_xyz, d.init_vel = _d(x0), _d(v0)
        d.rho, d.E, d.nu, d.per_element = float(rho), _d(E), _d(nu), int(E.size > 1)
        d.n_dirichlet, d.dirichlet_ids = ids.size, _i(ids)
        d.dt = float(dt)
        d.gravity[:] = [float(g) for g in gravity]
        d.precision = int(precision)
        p = None
        if params is not None:
            p = ppn_params_default()
            for k, v in params.items():
                setattr(p, k, v)
            d.params = C.pointer(p)
        sid = C.c_int32()
        _check(_abi.lib().ppn_engine_add_scene(self._h, C.byref(d), C.byref(sid)))
        return sid.value

    def add_scene(self, sc, precision=PPN_FP64, params=None):
        """Register a ``scenes.Scene`` (mesh, material, time step, constrained ids, initial state)."""
        kw = dict(stop_mode=PPN_STOP_VEL if sc.stop_mode == "vel" else PPN_STOP_GRAD_REL,
                  stop_tol=sc.stop_tol)
        kw.update(params or {})
        return self.ppn_engine_add_scene(sc.X, sc.tets, sc.E, sc.nu, sc.rho, sc.dt, sc.gravity,
                                         sc.dirichlet_ids, precision, kw, sc.x0, sc.v0)

    def ppn_engine_scene_footprint(self, scene_id):
        b = C.c_int64()
        _check(_abi.lib().ppn_engine_scene_footprint(self._h, int(scene_id), C.byref(b)))
        return b.value

    def ppn_engine_submit(self, scene_id, mode, targets):
        t = _f64(targets)
        rid = C.c_int64()
        _check(_abi.lib().ppn_engine_submit(self._h, int(scene_id), MODES[mode], _d(t), C.byref(rid)))
        return rid.value

    def ppn_engine_wait(self, request_id):
        st = C.c_int()
        stats = ppn_step_stats()
        lat, que = C.c_double(), C.c_double()
        _check(_abi.lib().ppn_engine_wait(self._h, int(request_id), C.byref(st), C.byref(stats),
                                           C.byref(lat), C.byref(que)))
        d = stats.as_dict()
        d["status"] = STATUS.get(st.value, st.value)
        if st.value < 0:
            msg = _abi.lib().ppn_last_error(None)
            d["error"] = msg.decode() if msg else ""
        d["latency_ms"], d["queue_ms"] = lat.value, que.value
        return d

    def ppn_engine_get_state(self, scene_id, n_verts):
        x = np.empty((n_verts, 3))
        v = np.empty((n_verts, 3))
        _check(_abi.lib().ppn_engine_get_state(self._h, int(scene_id), _d(x), _d(v)))
        return x, v

    def ppn_engine_set_pcg_batching(self, enable=True):
        _check(_abi.lib().ppn_engine_set_pcg_batching(self._h, int(bool(enable))))

    def ppn_engine_set_batching(self, pcg=True, evaluation=False):
        """Shared launches across scenes: PCG solves, and with evaluation=True the
        per-iteration evaluation and line-search phases too."""
        flags = (_abi.PPN_BATCH_PCG if pcg else 0) | (_abi.PPN_BATCH_EVAL if evaluation else 0)
        _check(_abi.lib().ppn_engine_set_batching(self._h, flags))

    def ppn_engine_get_info(self):
        i = ppn_engine_info()
        _check(_abi.lib().ppn_engine_get_info(self._h, C.byref(i)))
        return i.as_dict()


def scene_from(sc, stream=None, params=None, trace=False, precision=PPN_FP64):
    """A Scene loaded with a ``scenes.Scene`` description (mesh, material, dt, first targets)."""
    s = Scene(stream=stream, precision=precision)
    s.ppn_load_mesh(sc.X, sc.tets, sc.x0)
    s.ppn_set_material(sc.rho, sc.E, sc.nu)
    s.ppn_set_time_step(sc.dt, sc.gravity)
    kw = dict(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol)
    if params:
        kw.update(params)
    s.ppn_set_params(**kw)
    if np.any(sc.v0 != 0.0):
        s.ppn_set_state(sc.x0, sc.v0)
    s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(1))
    if trace:
        s.ppn_set_trace(True)
    return s


def run_steps(s, sc, mode, n_steps, first_step=1, callback=None):
    """Advance ``n_steps`` time steps, moving the Dirichlet targets of ``sc`` each step."""
    stats = []
    for n in range(first_step, first_step + n_steps):
        s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(n))
        stats.append(s.ppn_newton_step(mode))
        if callback is not None:
            callback(n, s, stats[-1])
    return stats
