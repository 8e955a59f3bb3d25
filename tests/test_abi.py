"""The C-ABI library loads and exports every entry point include/arb.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2107_10800_amd import arb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "arb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(arb_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_symbols():
    assert sorted(arb.SYMBOLS) == declared()


def test_library_exports_every_symbol():
    if not os.path.exists(arb.LIB_PATH):
        pytest.fail("libarb.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(arb.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_bad_options_rejected_before_device():
    lib = arb.load()
    for kw in (dict(a=-1.0), dict(eta=0.0), dict(tol=0.0), dict(restart=0), dict(restart=1000),
               dict(precision=7), dict(precond=9), dict(precond=4), dict(max_iter=0),
               dict(pair_kernel=4), dict(graphs=2), dict(model=2),
               # single-blob bodies: unbounded, exact or no preconditioner
               dict(model=1, wall=1), dict(model=1, precond=2),
               # fast product: 2..8 points per direction, levels 0..16, leaf >= 0
               dict(pair_kernel=3, fmm_order=1), dict(pair_kernel=3, fmm_order=9),
               dict(fmm_levels=-1), dict(fmm_levels=17), dict(fmm_leaf=-1),
               # left or right preconditioning only; one-launch small cycles on or
               # off; bounded last refinement correction on or off
               dict(left_precond=2), dict(left_precond=-1), dict(small_cycle=2),
               dict(small_cycle=-1), dict(refine_final=2), dict(refine_final=-1)):
        base = dict(device=0, precision=0, wall=0, eta=1.0, a=1.0, tol=1e-8, restart=50,
                    max_iter=100, precond=1, slices=0, pair_kernel=0)
        base.update(kw)
        opt = arb.arb_options(**base)
        h = ctypes.c_void_p()
        assert lib.arb_create(ctypes.byref(h), ctypes.byref(opt)) == arb.ARB_E_ARG
        assert not h.value
    assert lib.arb_create(None, None) == arb.ARB_E_ARG


def test_null_context_calls_are_errors():
    lib = arb.load()
    assert lib.arb_set_state(None, None, None) == arb.ARB_E_ARG
    assert lib.arb_solve(None, None, None, None, None, None, None, None) == arb.ARB_E_ARG
    assert lib.arb_step_euler_arms(None, None, None, 0.1, 0.0, 1e-10, 10, 0, None, None, None,
                                   None, None) == arb.ARB_E_ARG
    assert lib.arb_step_midpoint_arms(None, None, None, 0.1, 0.0, 1e-10, 10, 0, None, None,
                                      None, None, None, None) == arb.ARB_E_ARG
    assert lib.arb_last_error(None) == b"null context"
