"""CPU-side checks of the C-ABI library: it loads, exports every entry point
the header declares, and its host-only helpers agree with the paper."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import synth
from paper_2604_25378_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "yand.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(yand_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libyand.so is not built (run __graft_entry__.build())")
    return binding.load()


def test_header_symbols_exported(lib):
    names = _declared()
    assert "yand_mvsk_solve" in names and "yand_hvp" in names
    assert "yand_mvsk_solve_R" in names and "yand_warmstart_train" in names
    for name in names:
        assert hasattr(lib, name), name


def test_certified_convex_matches_paper(lib, golden_dir):
    rows = np.atleast_2d(np.loadtxt(f"{golden_dir}/crra_calibration.txt"))
    for g, *cv in rows:
        assert binding.is_certified_convex(cv)
    for g in (0.5, 2.0, 4.0, 10.0):
        c = synth.crra_coefficients(g)
        assert binding.is_certified_convex(c) == O.certified_convex(c)
    assert not binding.is_certified_convex([10, 1, 10, 1])
    assert not binding.is_certified_convex([1, 1, 1, 0])


def test_default_opts_follow_parameter_table(lib):
    o = binding.default_opts()
    assert (o.solver, o.max_iter, o.eps, o.tau) == (0, 300, 1e-8, 1e-8)
    lg = binding.default_opts(large=True)
    assert (lg.solver, lg.max_iter, lg.max_elapsed) == (1, 40, 60.0)
    assert (lg.krylov_tol, lg.krylov_maxit, lg.regularization) == (1e-3, 15, 1e-4)
    assert lg.restart_max_iter == 120 and lg.stall_recovery == 1
    # projected trial step 0.05 in both configurations
    assert o.eta == 0.05 and lg.eta == 0.05
    assert o.linesearch == 0 and lg.linesearch == 0   # exact quartic rule


def test_simplex_entry_points_reject_bad_arguments_without_device(lib):
    p = C.c_void_p(8)
    assert lib.yand_project_simplex(None, 4, 0.0, p) == -1
    assert lib.yand_project_simplex(p, 0, 0.0, p) == -1
    assert lib.yand_project_simplex(p, 4, 0.25, p) == -1   # tau >= 1/n
    assert lib.yand_project_simplex(p, 4, -1e-9, p) == -1
    k = C.c_double()
    assert lib.yand_kkt_residual(None, (C.c_double * 4)(1, 1, 1, 1), p, 0.0, C.byref(k)) == -1
    prof = (C.c_double * 3)(1, 1, 10)
    assert lib.yand_return_floor(None, prof, 0.5, None, 40, None, None, None,
                                 p, None, None) == -1


def test_create_rejects_bad_arguments_without_device(lib):
    h = C.c_void_p()
    # null returns / bad sizes are rejected before any device work
    assert lib.yand_create(None, 10, 4, 4, 0, None, C.byref(h)) == -1
    assert lib.yand_create(C.c_void_p(8), 1, 4, 4, 0, None, C.byref(h)) == -1
    assert lib.yand_create(C.c_void_p(8), 10, 4, 3, 0, None, C.byref(h)) == -1
    assert lib.yand_create(C.c_void_p(8), 10, 4, 4, 7, None, C.byref(h)) == -1
    assert h.value is None


def test_mlp_entry_points_reject_bad_arguments_without_device(lib):
    o = binding.default_mlp_opts()
    assert (o.hidden, o.layers, o.epochs, o.lr) == (512, 4, 2000, 1e-3)
    h = C.c_void_p()
    assert lib.yand_mlp_create(0, 5, 8, 2, 0, None, C.byref(h)) == -1
    assert lib.yand_mlp_create(4, 5, 0, 2, 0, None, C.byref(h)) == -1
    assert lib.yand_mlp_create(4, 5, 8, 0, 0, None, C.byref(h)) == -1
    assert lib.yand_mlp_create(4, 5, 8, 2, 0, None, None) == -1
    assert h.value is None
    assert lib.yand_mlp_num_params(None) == -1
    assert lib.yand_mlp_forward(None, 1, C.c_void_p(8), C.c_void_p(8)) == -1
    assert lib.yand_mlp_adam_step(None, None, 1e-3) == -1
    assert lib.yand_mlp_destroy(None) == 0
    assert lib.yand_reduced_coords(0, 5, C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.yand_from_reduced(3, 1, C.c_void_p(8), C.c_void_p(8), None) == -1
    out = C.c_void_p()
    assert lib.yand_warmstart_train(None, 4, None, None, None, None,
                                    C.byref(out), None) == -1
    assert out.value is None
    assert lib.yand_warmstart_predict(None, None, 1, None, None, None, None,
                                      None) == -1


def test_autotune_rejects_null_context(lib):
    assert lib.yand_autotune(None, None) == -1
    assert lib.yand_tuning(None, None, None) == -1


def test_noalloc_refuses_oversized_instances_without_device(lib):
    """The allocation-free solve checks the instance against its fixed
    scratch array before any device call or read of R."""
    out = C.c_void_p(16)
    R = C.c_void_p(16)
    rc = lib.yand_mvsk_solve_R_noalloc(R, 12000, 2000, 1.0, 1.0, 1.0, 1.0,
                                       None, out)
    assert rc == -7
    assert lib.yand_mvsk_solve_R_noalloc(None, 500, 12, 1.0, 1.0, 1.0, 1.0,
                                         None, out) == -1
