"""The C-ABI library builds, loads and exports every entry point that
include/rgdbek.h declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2509_19267_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgdbek.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rgdbek_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["rgdbek_create", "rgdbek_solve", "rgdbek_destroy",
                 "rgdbek_status_string", "rgdbek_last_error",
                 "rgdbek_solve_adjoint", "rgdbek_grad_pattern",
                 "rgdbek_select"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(B.SIGNATURES)


def declared_arities():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for name, args in re.findall(r"\b(rgdbek_[a-z_]+)\s*\(([^)]*)\)\s*;", text):
        args = args.strip()
        out[name] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_header_arity():
    ar = declared_arities()
    assert len(ar) >= 12
    for name, n in ar.items():
        assert len(B.SIGNATURES[name][1]) == n, name


def test_struct_layouts_match_header_sizes():
    # int64 x3 + int32 x2 + 3 pointers
    assert ctypes.sizeof(B.Matrix) == 3 * 8 + 2 * 4 + 3 * 8
    assert ctypes.sizeof(B.Info) == 8 + 8 + 8 + 4 + 4 + 8


def test_params_default_and_status_strings():
    lib = B.load()
    p = B.Params()
    assert lib.rgdbek_params_default(ctypes.byref(p)) == B.OK
    assert p.eta == 0.5 and p.tol == 1e-8 and p.max_iter == 10000
    assert p.stop == B.STOP_ERR_REF and p.flags & B.FLAG_GRAPH
    assert lib.rgdbek_params_default(None) == B.ERR_INVALID_ARG
    for s in range(7):
        assert lib.rgdbek_status_string(s)
    assert lib.rgdbek_status_string(99) == b"unknown status"


def test_create_rejects_bad_arguments_before_touching_the_device():
    lib = B.load()
    p = B.Params()
    lib.rgdbek_params_default(ctypes.byref(p))
    h = ctypes.c_void_p()
    assert lib.rgdbek_create(None, ctypes.byref(p), None, ctypes.byref(h)) == B.ERR_INVALID_ARG
    m = B.Matrix()
    m.m, m.n, m.layout, m.value_type = 0, 5, B.DENSE_ROW_MAJOR, B.F64
    m.values = ctypes.c_void_p(1)
    assert lib.rgdbek_create(ctypes.byref(m), ctypes.byref(p), None, ctypes.byref(h)) == B.ERR_INVALID_ARG
    m.m, m.layout = 5, 7
    assert lib.rgdbek_create(ctypes.byref(m), ctypes.byref(p), None, ctypes.byref(h)) == B.ERR_INVALID_ARG
    m.layout, m.values = B.CSR, ctypes.c_void_p(1)
    m.row_ptr = None
    assert lib.rgdbek_create(ctypes.byref(m), ctypes.byref(p), None, ctypes.byref(h)) == B.ERR_INVALID_ARG
    assert b"CSR" in lib.rgdbek_last_error(None)
    assert lib.rgdbek_create(ctypes.byref(m), ctypes.byref(p), None, None) == B.ERR_INVALID_ARG
    assert lib.rgdbek_destroy(None) == B.OK
    assert lib.rgdbek_solve(None, None, None, None, None) == B.ERR_INVALID_ARG
    cnt = ctypes.c_int64()
    assert lib.rgdbek_select(None, 10, 2, 0.0, 0, 0, 0, 0, 0, None, ctypes.byref(cnt), None) == B.ERR_INVALID_ARG
    assert lib.rgdbek_apply(None, 0, None, None, None, None) == B.ERR_INVALID_ARG


def test_product_path_has_no_fallback():
    # the package refuses to work without the built library
    import importlib
    mod = importlib.import_module("paper_2509_19267_amd._binding")
    saved = mod._lib, mod.LIB_PATH
    try:
        mod._lib = None
        mod.LIB_PATH = "/nonexistent/librgdbek.so"
        with pytest.raises(RuntimeError):
            mod.load()
    finally:
        mod._lib, mod.LIB_PATH = saved


def test_block_diagonal_concatenation():
    import numpy as np
    import scipy.sparse as sp
    import workloads
    from paper_2509_19267_amd import block_diagonal
    ps = workloads.laplacian_batch(count=4, n_min=60, n_max=300, seed=3)
    rp, ci, v, ro, co = block_diagonal([p.a for p in ps])
    a = sp.csr_matrix((v, ci, rp), shape=(ro[-1], co[-1]))
    want = sp.block_diag([p.a for p in ps]).tocsr()
    assert abs(a - want).max() == 0.0
    assert rp.dtype == np.int64 and ci.dtype == np.int32
    for s in range(4):
        blk = a[ro[s]:ro[s + 1]]
        assert blk.indices.min() >= co[s] and blk.indices.max() < co[s + 1]
