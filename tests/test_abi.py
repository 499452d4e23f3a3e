"""The C-ABI library loads on a machine without a GPU and exports every function that
include/trsyl.h declares; the host-only calls (defaults, workspace sizes, argument checks) work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trsyl.h")
LIB = os.path.join(ROOT, "paper_1905_10574_amd", "libtrsyl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(trsyl_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libtrsyl.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["trsyl_robust", "trsyl_workspace_size", "trsyl_robust_adjoint", "trsyl_grad",
                 "trsyl_robust_batched", "trsyl_residual", "trsyl_default_opts", "trsyl_version"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls(lib):
    import paper_1905_10574_amd as T
    o = T.Opts()
    lib.trsyl_default_opts(ctypes.byref(o))
    assert o.tile_m == 128 and o.tile_n == 128 and o.precision == 0 and o.scheduler == 0
    lib.trsyl_workspace_size.restype = ctypes.c_size_t
    lib.trsyl_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(T.Opts)]
    assert lib.trsyl_workspace_size(1000, 700, ctypes.byref(o)) > 0
    assert lib.trsyl_workspace_size(-1, 7, ctypes.byref(o)) == 0
    bad = T.Opts()
    lib.trsyl_default_opts(ctypes.byref(bad))
    bad.tile_m = 8                                  # below the supported range
    assert lib.trsyl_workspace_size(100, 100, ctypes.byref(bad)) == 0
    lib.trsyl_version.restype = ctypes.c_char_p
    assert lib.trsyl_version().startswith(b"trsyl")


def test_argument_errors_are_reported_without_a_device(lib):
    """Invalid arguments are rejected on the host before anything is enqueued."""
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.trsyl_robust.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, P, P, P, P, ctypes.c_size_t, P]
    dummy = ctypes.c_void_p(256)
    assert lib.trsyl_robust(-1, 4, dummy, 4, dummy, 4, dummy, 4, dummy, None, dummy, None, dummy, 1 << 20, None) == -1
    assert lib.trsyl_robust(4, 4, None, 4, dummy, 4, dummy, 4, dummy, None, dummy, None, dummy, 1 << 20, None) == -3
    assert lib.trsyl_robust(4, 4, dummy, 3, dummy, 4, dummy, 4, dummy, None, dummy, None, dummy, 1 << 20, None) == -4
    assert lib.trsyl_robust(4, 4, dummy, 4, dummy, 4, dummy, 4, None, None, dummy, None, dummy, 1 << 20, None) == -9
    assert lib.trsyl_robust(4, 4, dummy, 4, dummy, 4, dummy, 4, dummy, None, dummy, None, dummy, 8, None) == -14


def test_general_form_argument_errors(lib):
    """trsyl_robust_general reports argument i as -i on the host (LAPACK convention)."""
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.trsyl_robust_general.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int32, I64, I64, P, I64,
                                         P, I64, P, I64, P, P, P, P, P, ctypes.c_size_t, P]
    d = ctypes.c_void_p(256)

    def call(ta=b"N", tb=b"N", sg=1, m=4, n=4, A=d, lda=4, B=d, ldb=4, C=d, ldc=4, e=d, info=d, ws=1 << 24):
        return lib.trsyl_robust_general(ta, tb, sg, m, n, A, lda, B, ldb, C, ldc, e, None, info, None, d, ws, None)

    assert call(ta=b"X") == -1
    assert call(tb=b"Q") == -2
    assert call(sg=0) == -3 and call(sg=2) == -3
    assert call(m=-1) == -4
    assert call(n=-2) == -5
    assert call(A=None) == -6
    assert call(lda=3) == -7
    assert call(B=None) == -8
    assert call(ldb=2) == -9
    assert call(C=None) == -10
    assert call(ldc=1) == -11
    assert call(e=None) == -12
    assert call(info=None) == -14
    assert call(ws=8) == -17


def test_bartels_stewart_argument_errors(lib):
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.trsyl_bartels_stewart.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, I64, P, I64, P, P, P, P, P,
                                          ctypes.c_size_t, P]
    d = ctypes.c_void_p(256)

    def call(m=4, n=4, U=d, ldu=4, At=d, ldat=4, V=d, ldv=4, Bt=d, ldbt=4, C=d, ldc=4, e=d, info=d, ws=1 << 24):
        return lib.trsyl_bartels_stewart(m, n, U, ldu, At, ldat, V, ldv, Bt, ldbt, C, ldc, e, None, info, None,
                                         d, ws, None)

    assert call(m=-1) == -1 and call(n=-1) == -2
    assert call(U=None) == -3 and call(ldu=2) == -4
    assert call(At=None) == -5 and call(ldat=3) == -6
    assert call(V=None) == -7 and call(ldv=1) == -8
    assert call(Bt=None) == -9 and call(ldbt=3) == -10
    assert call(C=None) == -11 and call(ldc=3) == -12
    assert call(e=None) == -13 and call(info=None) == -15
    assert call(ws=8) == -18


def test_sync_result_argument_errors(lib):
    P = ctypes.c_void_p
    lib.trsyl_sync_result.argtypes = [P, P, P, P, P, P, P]
    d = ctypes.c_void_p(256)
    h64, hd, h32 = ctypes.c_int64(0), ctypes.c_double(0.0), ctypes.c_int32(0)
    assert lib.trsyl_sync_result(None, d, d, ctypes.byref(h64), ctypes.byref(hd), ctypes.byref(h32), None) == -1
    assert lib.trsyl_sync_result(d, None, d, ctypes.byref(h64), ctypes.byref(hd), ctypes.byref(h32), None) == -2
    assert lib.trsyl_sync_result(d, d, None, ctypes.byref(h64), ctypes.byref(hd), ctypes.byref(h32), None) == -3
    assert lib.trsyl_sync_result(d, d, d, None, ctypes.byref(hd), ctypes.byref(h32), None) == -4
    assert lib.trsyl_sync_result(d, d, d, ctypes.byref(h64), ctypes.byref(hd), None, None) == -6


def test_colmajor_fresh_never_aliases_the_callers_tensor():
    """A column-major float64 operand is passed through without a copy, except for operands the
    library overwrites (C / W), which always get a buffer of their own."""
    import torch
    import paper_1905_10574_amd as T
    X = torch.arange(12, dtype=torch.float64).reshape(3, 4).t().contiguous().t()   # column-major
    S = T.colmajor(X, torch.device("cpu"))
    assert S.data_ptr() == X.data_ptr() and torch.equal(S.t(), X)
    F = T.colmajor(X, torch.device("cpu"), fresh=True)
    assert F.data_ptr() != X.data_ptr() and torch.equal(F.t(), X)
    R = torch.arange(12, dtype=torch.float64).reshape(3, 4)                     # row-major
    F2 = T.colmajor(R, torch.device("cpu"), fresh=True)
    assert F2.data_ptr() != R.data_ptr() and torch.equal(F2.t(), R)


def test_noalloc_rejects_without_a_device(lib):
    """trsyl_robust_noalloc checks its arguments and whether the problem's state fits its fixed
    array on the host, before any device call: a problem too large for TRSYL_NOALLOC_BYTES gives
    TRSYL_ENOSPACE, the precision form is refused (-12), bad sizes give their argument index."""
    import paper_1905_10574_amd as T
    L = T.lib()
    o = T.make_opts()
    fake = 256                                   # never dereferenced on these paths
    args = lambda m, n: (m, n, fake, max(1, m), fake, max(1, n), fake, max(1, m), fake, fake, fake)
    assert L.trsyl_robust_noalloc(*args(40000, 40000), ctypes.byref(o), None) == T.ENOSPACE
    assert L.trsyl_robust_noalloc(*args(-1, 5), ctypes.byref(o), None) == -1
    p = T.make_opts(precision="fp32_refine")
    assert L.trsyl_robust_noalloc(*args(100, 100), ctypes.byref(p), None) == -12
    bad = T.make_opts()
    bad.tile_m = 8
    assert L.trsyl_robust_noalloc(*args(100, 100), ctypes.byref(bad), None) == -12
