"""The C ABI library builds, loads and exports every entry point declared in include/ppn.h;
host-side argument checking works without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ppn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppn_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ppn_scene_create", "ppn_load_mesh", "ppn_set_material", "ppn_set_time_step",
                 "ppn_set_dirichlet", "ppn_newton_step", "ppn_get_last_stats", "ppn_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2505_21013_amd import _abi
    lib = _abi.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(_abi.SIGNATURES), "binding table out of sync with the header"


def test_struct_layouts_match_header():
    from paper_2505_21013_amd import _abi
    # ppn_params: 5 doubles, 4 int32, 2 doubles, 2 int32, 1 double, 2 int32 = 96 bytes
    assert ctypes.sizeof(_abi.ppn_params) == 5 * 8 + 4 * 4 + 2 * 8 + 2 * 4 + 8 + 2 * 4
    assert ctypes.sizeof(_abi.ppn_step_stats) == 10 * 4 + 8 + 7 * 8 + 8 + 2 * 4
    assert ctypes.sizeof(_abi.ppn_iter_record) == 6 * 4 + 6 * 8


def test_defaults_follow_the_paper():
    from paper_2505_21013_amd import ppn_params_default
    p = ppn_params_default()
    assert (p.alpha, p.beta, p.eps_delta) == (0.5, 2.0, 1e-12)
    assert (p.eps_clamp, p.pcg_rtol, p.pdn_countdown, p.stop_tol) == (1e-8, 1e-4, 4, 1e-3)


def test_host_side_errors_without_gpu():
    from paper_2505_21013_amd import _abi
    lib = _abi.lib()
    h = ctypes.c_void_p()
    assert lib.ppn_scene_create(ctypes.byref(h), None, 7) == -1  # unknown precision, before touching HIP
    assert b"PPN_MIXED" in lib.ppn_last_error(None)
    assert lib.ppn_newton_step(None, 2, None) == -1
    assert b"NULL scene handle" in lib.ppn_last_error(None)
    assert lib.ppn_params_default(None) == -1
    assert b"out must not be NULL" in lib.ppn_last_error(None)
    assert lib.ppn_project_batch_dev(None, None, 4, 1e-8, None) == -1


def test_noalloc_limit_matches_header():
    from paper_2505_21013_amd import _abi
    src = open(os.path.join(ROOT, "include", "ppn.h")).read()
    assert int(re.search(r"#define PPN_NOALLOC_MAX_ELEMENTS (\d+)", src).group(1)) == _abi.PPN_NOALLOC_MAX_ELEMENTS
