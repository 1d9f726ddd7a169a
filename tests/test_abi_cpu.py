"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only entry points behave (no device work)."""
import ctypes as C
import os
import re

import pytest

from paper_1512_04629_amd import amg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "amg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z0-9_]+)\s*\(", text)) - {"amg_alloc_fn", "amg_free_fn"})


def test_header_and_binding_agree():
    assert header_functions() == sorted(amg.ABI_SYMBOLS)


def test_library_exports_every_symbol():
    lib = amg.load_library()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_defaults_and_status_strings():
    lib = amg.load_library()
    sp = amg.SetupParams()
    lib.amg_setup_params_default(C.byref(sp))
    assert (sp.theta, sp.max_coarse, sp.max_levels, sp.nu_pre, sp.nu_post) == (0.25, 49, 25, 1, 1)
    assert abs(sp.omega - 2.0 / 3.0) < 1e-16
    pp = amg.SolveParams()
    pp.zero_guess = 7
    lib.amg_solve_params_default(C.byref(pp))
    assert (pp.method, pp.rtol, pp.maxit, pp.k, pp.s, pp.rho_max, pp.gamma_min) == (1, 1e-8, 200, 3, 1, 0.5, 0.01)
    assert (pp.precision, pp.zero_guess) == (64, 0)
    for st in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert lib.amg_status_string(st)


def test_null_handle_and_bad_arguments_are_rejected_without_a_device():
    lib = amg.load_library()
    assert lib.amg_sparsify(None, 0.1, 2) == -7
    assert lib.amg_solve(None, None, None, None, None, None) == -7
    out = C.c_void_p()
    # n <= 0 and NULL arrays are rejected before any device call
    assert lib.amg_setup_from_csr(0, None, None, None, None, None, amg.ALLOC_FN(), amg.FREE_FN(),
                                  None, C.byref(out)) == -1
    assert out.value is None
    # device setup: sizes, NULL arrays and the coarsening are checked first
    fake = C.c_void_p(16)
    assert lib.amg_setup_device(0, 0, fake, fake, fake, None, 0, 0, None, amg.ALLOC_FN(), amg.FREE_FN(),
                                None, C.byref(out)) == -1
    assert lib.amg_setup_device(10, 5, fake, fake, fake, None, 0, 0, None, amg.ALLOC_FN(), amg.FREE_FN(),
                                None, C.byref(out)) == -1
    assert lib.amg_setup_device(10, 28, fake, fake, fake, None, 2, 0, None, amg.ALLOC_FN(), amg.FREE_FN(),
                                None, C.byref(out)) == -1
    assert lib.amg_setup_device(10, 28, None, fake, fake, None, 1, 0, None, amg.ALLOC_FN(), amg.FREE_FN(),
                                None, C.byref(out)) == -1
    assert out.value is None
    lib.amg_destroy(None)


def test_library_is_gfx950_only():
    so = open(amg.LIB_PATH, "rb").read()
    assert b"gfx950" in so
