"""Plain FP64 CPU oracle for the robust triangular Sylvester solve (arXiv 1905.10574, Sec. 2).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this package.  It shares no code with the GPU library (paper_1905_10574_amd) and
never imports it.  The arithmetic lives in oracle.c (plain C, no BLAS); this module builds it
with gcc and marshals numpy arrays.

All matrices are float64, column-major.  A returned exponent e means alpha = 2^-e.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None

OMEGA = 2.0 ** 1022
RC_OK, RC_PERTURBED, RC_BAD_STRUCTURE, RC_BAD_INPUT = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (plain -O2, OpenMP for the optional tile parallelism)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_protect_update.argtypes = [ctypes.c_double] * 3
        lib.orc_protect_update.restype = ctypes.c_int
        lib.orc_protect_division.argtypes = [ctypes.c_double] * 2
        lib.orc_protect_division.restype = ctypes.c_int
        lib.orc_block_starts.argtypes = [i64, dp, i64, i64p]
        lib.orc_block_starts.restype = i64
        lib.orc_tile_offsets.argtypes = [i64, dp, i64, i64, i64p]
        lib.orc_tile_offsets.restype = i64
        lib.orc_small_solve.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, dp, i64, dp, i64,
                                        ctypes.c_double, ip, ip]
        lib.orc_small_solve.restype = None
        lib.orc_nonrobust_syl.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.orc_nonrobust_syl.restype = ctypes.c_int
        lib.orc_robust_syl_driver.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i64p]
        lib.orc_robust_syl_driver.restype = ctypes.c_int
        lib.orc_drsylv.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i64, i64, ctypes.c_int, i64p]
        lib.orc_drsylv.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i64, i64, ctypes.c_int, i64p]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_relres.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i64, dp, i64]
        lib.orc_relres.restype = ctypes.c_double
        lib.orc_residual_rows.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i64, dp, i64,
                                          ctypes.c_int, i64, i64p, dp]
        lib.orc_residual_rows.restype = None
        lib.orc_smin.argtypes = [i64, i64, dp, i64, dp, i64]
        lib.orc_smin.restype = ctypes.c_double
        _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    return np.asfortranarray(np.asarray(x, dtype=np.float64))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


# ---- primitives --------------------------------------------------------------------------

def protect_update(c: float, a: float, y: float) -> int:
    """ProtectUpdate: s with 2^-s (c + a*y) <= Omega (Sec. 2.1)."""
    return _load().orc_protect_update(c, a, y)


def protect_division(b: float, t: float) -> int:
    """ProtectDivision: smallest s with 2^-s |b| <= |t| Omega (Sec. 2.1)."""
    return _load().orc_protect_division(b, t)


def block_starts(T) -> list[int]:
    T = _f64(T)
    n = T.shape[0]
    out = np.zeros(n + 1, dtype=np.int64)
    nb = _load().orc_block_starts(n, _dp(T), _ld(T), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if nb < 0:
        raise ValueError("two consecutive nonzero subdiagonal entries")
    return [int(x) for x in out[:nb]]


def tile_offsets(T, t: int) -> list[int]:
    T = _f64(T)
    n = T.shape[0]
    out = np.zeros(n // max(t, 1) + 2, dtype=np.int64)
    cnt = _load().orc_tile_offsets(n, _dp(T), _ld(T), t, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return [int(x) for x in out[:cnt + 1]]


def small_solve(A11, B11, R, smin: float = 2.0 ** -1022):
    """Robust A11 Z + Z B11 = beta R for 1x1/2x2 blocks.  Returns (Z, s_beta, perturbed)."""
    A11, B11, Z = _f64(A11), _f64(B11), _f64(R).copy(order="F")
    r, c = A11.shape[0], B11.shape[0]
    sb, pt = ctypes.c_int(0), ctypes.c_int(0)
    _load().orc_small_solve(r, c, _dp(A11), _ld(A11), _dp(B11), _ld(B11), _dp(Z), _ld(Z), smin,
                            ctypes.byref(sb), ctypes.byref(pt))
    return Z, sb.value, pt.value


# ---- solvers ------------------------------------------------------------------------------

def nonrobust_syl(A, B, C) -> np.ndarray:
    """Algorithm 1, no scaling (may overflow)."""
    A, B = _f64(A), _f64(B)
    Y = _f64(C).copy(order="F")
    m, n = Y.shape
    with np.errstate(all="ignore"):
        rc = _load().orc_nonrobust_syl(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(Y), _ld(Y))
    if rc:
        raise ValueError(f"nonrobust_syl rc={rc}")
    return Y


def robust_syl(A, B, C):
    """Algorithm 2 on the whole problem.  Returns (Y, e, rc) with A Y + Y B = 2^-e C."""
    A, B = _f64(A), _f64(B)
    Y = _f64(C).copy(order="F")
    m, n = Y.shape
    e = ctypes.c_int64(0)
    rc = _load().orc_robust_syl_driver(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(Y), _ld(Y), ctypes.byref(e))
    return Y, e.value, rc


def drsylv(A, B, C, tile_m: int = 64, tile_n: int | None = None, threads: int = 1):
    """Algorithm 4 (tiled, per-tile scales).  Returns (Y, e, rc) with A Y + Y B = 2^-e C."""
    A, B = _f64(A), _f64(B)
    Y = _f64(C).copy(order="F")
    m, n = Y.shape
    e = ctypes.c_int64(0)
    tn = tile_m if tile_n is None else tile_n
    rc = _load().orc_drsylv(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(Y), _ld(Y), tile_m, tn,
                            threads, ctypes.byref(e))
    return Y, e.value, rc


def adjoint(A, B, W, tile_m: int = 64, tile_n: int | None = None, threads: int = 1):
    """A^T G + G B^T = 2^-e W.  Returns (G, e, rc)."""
    A, B = _f64(A), _f64(B)
    G = _f64(W).copy(order="F")
    m, n = G.shape
    e = ctypes.c_int64(0)
    tn = tile_m if tile_n is None else tile_n
    rc = _load().orc_adjoint(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(G), _ld(G), tile_m, tn,
                             threads, ctypes.byref(e))
    return G, e.value, rc


def relres(A, B, Y, e: int, C) -> float:
    """Eq. (9) relative residual, scale-safe, long-double sums."""
    A, B, Y, C = _f64(A), _f64(B), _f64(Y), _f64(C)
    m, n = Y.shape
    return _load().orc_relres(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(Y), _ld(Y), int(e), _dp(C), _ld(C))


def residual_rows(A, B, Y, e: int, C, rows, shift: int):
    """Sums over the listed rows of |R|^2, |Y 2^-shift|^2, |alpha 2^-shift C|^2."""
    A, B, Y, C = _f64(A), _f64(B), _f64(Y), _f64(C)
    m, n = Y.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros(3)
    _load().orc_residual_rows(m, n, _dp(A), _ld(A), _dp(B), _ld(B), _dp(Y), _ld(Y), int(e), _dp(C),
                              _ld(C), int(shift), len(rows),
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    return out


def smin(A, B) -> float:
    A, B = _f64(A), _f64(B)
    return _load().orc_smin(A.shape[0], B.shape[0], _dp(A), _ld(A), _dp(B), _ld(B))
