"""ctypes declarations of the C ABI in include/ppn.h (argument marshalling only)."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libppn.so")

PPN_PN, PPN_PDN, PPN_PPN = 0, 1, 2
MODES = {"PN": PPN_PN, "PDN": PPN_PDN, "PPN": PPN_PPN}
PPN_FP64, PPN_MIXED = 0, 1
PPN_STOP_VEL, PPN_STOP_GRAD_REL = 0, 1
PPN_ORDER_PENCIL, PPN_ORDER_MORTON = 0, 1
PPN_NOALLOC_MAX_ELEMENTS = 4096  # include/ppn.h
PPN_BATCH_PCG, PPN_BATCH_EVAL = 1, 2
STATUS = {0: "PPN_OK", -1: "PPN_ERR_ARG", -2: "PPN_ERR_MESH", -3: "PPN_ERR_OOM", -4: "PPN_ERR_DEVICE",
          -5: "PPN_ERR_STATE", 1: "PPN_WARN_NOT_CONVERGED", 2: "PPN_WARN_LS_FAIL"}


class ppn_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("eps_delta", C.c_double),
                ("eps_clamp", C.c_double), ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int32),
                ("pdn_countdown", C.c_int32), ("stop_mode", C.c_int32), ("newton_maxit", C.c_int32),
                ("stop_tol", C.c_double), ("armijo_c", C.c_double), ("ls_maxit", C.c_int32),
                ("eig_mirror", C.c_int32), ("k_dirichlet", C.c_double), ("pcg_load_mode", C.c_int32),
                ("use_graphs", C.c_int32)]


class ppn_step_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("solves", C.c_int32),
                ("indefinite_solves", C.c_int32), ("inner_rounds", C.c_int32),
                ("ls_backtracks", C.c_int32), ("safety_events", C.c_int32), ("converged", C.c_int32),
                ("ls_fail", C.c_int32), ("skipped_solves", C.c_int32), ("projected", C.c_int64),
                ("res0_l2", C.c_double), ("res_l2", C.c_double), ("res_inf", C.c_double),
                ("ms_total", C.c_double), ("ms_eig", C.c_double), ("ms_pcg", C.c_double),
                ("ms_spmv", C.c_double), ("n_spmv", C.c_int64),
                ("refine_rounds", C.c_int32), ("reserved1", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ppn_iter_record(C.Structure):
    _fields_ = [("k", C.c_int32), ("first_ind", C.c_int32), ("first_iters", C.c_int32),
                ("rounds", C.c_int32), ("n_projected", C.c_int32), ("last_ind", C.c_int32),
                ("g_l2", C.c_double), ("g_inf", C.c_double), ("delta_in", C.c_double),
                ("delta_out", C.c_double), ("dx_inf", C.c_double), ("gamma", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ppn_scene_desc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("rest_xyz", C.POINTER(C.c_double)),
                ("tets", C.POINTER(C.c_int32)), ("init_xyz", C.POINTER(C.c_double)),
                ("init_vel", C.POINTER(C.c_double)), ("rho", C.c_double),
                ("E", C.POINTER(C.c_double)), ("nu", C.POINTER(C.c_double)),
                ("per_element", C.c_int32), ("n_dirichlet", C.c_int32),
                ("dirichlet_ids", C.POINTER(C.c_int32)), ("dt", C.c_double),
                ("gravity", C.c_double * 3), ("precision", C.c_int32), ("reserved0", C.c_int32),
                ("params", C.POINTER(ppn_params))]


class ppn_engine_info(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("resident_bytes", C.c_int64), ("admissions", C.c_int64),
                ("evictions", C.c_int64), ("resident_scenes", C.c_int32), ("n_scenes", C.c_int32),
                ("n_workers", C.c_int32), ("pending", C.c_int32), ("pcg_batches", C.c_int64),
                ("pcg_batched_solves", C.c_int64), ("eval_launches", C.c_int64),
                ("eval_batched_phases", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int32)
u8p = C.POINTER(C.c_uint8)
i64p = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every entry point of include/ppn.h
SIGNATURES = {
    "ppn_params_default": (C.c_int, [C.POINTER(ppn_params)]),
    "ppn_scene_create": (C.c_int, [C.POINTER(P), P, C.c_int32]),
    "ppn_scene_destroy": (C.c_int, [P]),
    "ppn_load_mesh": (C.c_int, [P, C.c_int32, dp, C.c_int32, ip, dp]),
    "ppn_set_material": (C.c_int, [P, C.c_double, dp, dp, C.c_int32]),
    "ppn_set_time_step": (C.c_int, [P, C.c_double, dp]),
    "ppn_set_dirichlet": (C.c_int, [P, C.c_int32, ip, dp]),
    "ppn_set_params": (C.c_int, [P, C.POINTER(ppn_params)]),
    "ppn_newton_step": (C.c_int, [P, C.c_int32, C.POINTER(ppn_step_stats)]),
    "ppn_get_positions": (C.c_int, [P, dp]),
    "ppn_get_positions_dev": (C.c_int, [P, P, P]),
    "ppn_get_state": (C.c_int, [P, dp, dp]),
    "ppn_set_state": (C.c_int, [P, dp, dp]),
    "ppn_get_last_stats": (C.c_int, [P, C.POINTER(ppn_step_stats)]),
    "ppn_scene_info": (C.c_int, [P, ip, ip, ip, i64p, i64p]),
    "ppn_last_error": (C.c_char_p, [P]),
    "ppn_set_trace": (C.c_int, [P, C.c_int32]),
    "ppn_set_profiling": (C.c_int, [P, C.c_int32]),
    "ppn_trace_count": (C.c_int, [P, ip]),
    "ppn_trace_get": (C.c_int, [P, C.c_int32, C.POINTER(ppn_iter_record), ip]),
    "ppn_eval_gradient": (C.c_int, [P, dp, dp]),
    "ppn_eval_element_hessians": (C.c_int, [P, dp, u8p, C.c_int32, ip, dp]),
    "ppn_eval_element_hessians_noalloc": (C.c_int, [P, dp, u8p, C.c_int32, ip, dp]),
    "ppn_eval_hessian": (C.c_int, [P, dp, u8p, ip, ip, dp]),
    "ppn_select": (C.c_int, [P, dp, C.c_double, u8p, u8p, ip]),
    "ppn_solve": (C.c_int, [P, dp, u8p, dp, ip, ip]),
    "ppn_debug_iterate": (C.c_int, [P, C.c_int32, dp, C.c_double, u8p, dp, ip]),
    "ppn_hessian_product": (C.c_int, [P, dp, u8p, dp, dp]),
    "ppn_energy_difference": (C.c_int, [P, dp, dp, C.c_int32, dp, dp]),
    "ppn_project_batch_dev": (C.c_int, [P, P, C.c_int64, C.c_double, P]),
    "ppn_locality_order": (C.c_int, [C.c_int32, dp, C.c_int32, ip, C.c_int32, ip, ip]),
    "ppn_engine_create": (C.c_int, [C.POINTER(P), C.c_int32, C.c_int64]),
    "ppn_engine_destroy": (C.c_int, [P]),
    "ppn_engine_add_scene": (C.c_int, [P, C.POINTER(ppn_scene_desc), ip]),
    "ppn_engine_scene_footprint": (C.c_int, [P, C.c_int32, i64p]),
    "ppn_engine_submit": (C.c_int, [P, C.c_int32, C.c_int32, dp, i64p]),
    "ppn_engine_wait": (C.c_int, [P, C.c_int64, C.POINTER(C.c_int), C.POINTER(ppn_step_stats), dp, dp]),
    "ppn_engine_get_state": (C.c_int, [P, C.c_int32, dp, dp]),
    "ppn_engine_get_info": (C.c_int, [P, C.POINTER(ppn_engine_info)]),
    "ppn_engine_set_pcg_batching": (C.c_int, [P, C.c_int32]),
    "ppn_engine_set_batching": (C.c_int, [P, C.c_int32]),
}

_lib = None


def lib():
    """The loaded libppn.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
