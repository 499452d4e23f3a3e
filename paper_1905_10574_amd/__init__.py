"""MI355X (gfx950) robust solver for the triangular Sylvester equation A Y + Y B = alpha C.

After Schwarz & Kjelgaard Mikkelsen, "Robust Task-Parallel Solution of the Triangular Sylvester
Equation" (arXiv 1905.10574).  Every step of the solve runs in the HIP library libtrsyl.so
(include/trsyl.h); this module only marshals torch tensors (device memory, streams) into the C
ABI.  There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["Opts", "lib", "solve", "solve_async", "adjoint", "grad", "residual", "solve_batched",
           "debug_protect_update", "debug_protect_division", "TrsylFunction", "workspace_size",
           "FP64", "FP32_REFINE", "SCHED_DAG", "SCHED_FRONTS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrsyl.so")

FP64, FP32_REFINE = 0, 1
SCHED_DAG, SCHED_FRONTS = 0, 1
_PREC = {"fp64": FP64, "fp32_refine": FP32_REFINE, FP64: FP64, FP32_REFINE: FP32_REFINE}
_SCHED = {"dag": SCHED_DAG, "fronts": SCHED_FRONTS, SCHED_DAG: SCHED_DAG, SCHED_FRONTS: SCHED_FRONTS}


class Opts(ctypes.Structure):
    _fields_ = [("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("scheduler", ctypes.c_int32),
                ("slabs", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("workers", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("profile_events", ctypes.c_void_p),
                ("trace", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def lib() -> ctypes.CDLL:
    """The loaded libtrsyl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_10574_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.trsyl_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.trsyl_default_opts.restype = None
        L.trsyl_version.restype = ctypes.c_char_p
        L.trsyl_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(Opts)]
        L.trsyl_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _P,
                                   ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P]
        L.trsyl_robust.restype = ctypes.c_int
        L.trsyl_adjoint_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(Opts)]
        L.trsyl_adjoint_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_adjoint.argtypes = L.trsyl_robust.argtypes
        L.trsyl_robust_adjoint.restype = ctypes.c_int
        L.trsyl_grad.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P,
                                 _P, _I64, _P, _I64, _P, _I64, _P]
        L.trsyl_grad.restype = ctypes.c_int
        L.trsyl_residual_workspace_size.argtypes = [_I64, _I64]
        L.trsyl_residual_workspace_size.restype = ctypes.c_size_t
        L.trsyl_residual.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P, _P,
                                     ctypes.c_size_t, _P]
        L.trsyl_residual.restype = ctypes.c_int
        L.trsyl_batched_workspace_size.argtypes = [ctypes.c_int32, _P, _P, ctypes.POINTER(Opts)]
        L.trsyl_batched_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_batched.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                           ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P]
        L.trsyl_robust_batched.restype = ctypes.c_int
        L.trsyl_debug_protect_update.argtypes = [ctypes.c_int32, _P, _P, _P]
        L.trsyl_debug_protect_update.restype = ctypes.c_int
        L.trsyl_debug_protect_division.argtypes = [ctypes.c_int32, _P, _P, _P]
        L.trsyl_debug_protect_division.restype = ctypes.c_int
        _lib = L
    return _lib


def make_opts(tile=None, tile_n=None, precision="fp64", scheduler="dag", slabs=0, workers=0,
              flags=0, max_sweeps=0, refine_tol=0.0) -> Opts:
    o = Opts()
    lib().trsyl_default_opts(ctypes.byref(o))
    if tile:
        o.tile_m = int(tile)
        o.tile_n = int(tile_n or tile)
    elif tile_n:
        o.tile_n = int(tile_n)
    o.precision = _PREC[precision]
    o.scheduler = _SCHED[scheduler]
    o.slabs = int(slabs)
    o.workers = int(workers)
    o.flags = int(flags)
    o.max_sweeps = int(max_sweeps)
    if refine_tol:
        o.refine_tol = float(refine_tol)
    return o


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def colmajor(X: torch.Tensor, device=None) -> torch.Tensor:
    """Column-major float64 copy on the device, returned as its transposed (row-major) storage
    tensor S with S.t() == X; S.data_ptr() is the column-major buffer with ld = X.shape[0]."""
    if not isinstance(X, torch.Tensor):
        X = torch.as_tensor(X)
    if device is None:
        device = X.device if X.is_cuda else torch.device("cuda")
    return X.to(device=device, dtype=torch.float64).t().contiguous()


def _aligned_workspace(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def workspace_size(m: int, n: int, opts: Opts) -> int:
    return int(lib().trsyl_workspace_size(m, n, ctypes.byref(opts)))


def solve_async(A, B, C, opts: Opts | None = None, *, workspace=None):
    """Enqueue the robust solve on the current stream.  A (m x m), B (n x n), C (m x n) tensors
    (any layout; copied to column-major float64 on the device).  Returns (Ys, e, scale, info)
    device tensors, with Ys the column-major storage (Y = Ys.t())."""
    opts = opts or make_opts()
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Yc = colmajor(C, dev)
    m, n = Yc.shape[1], Yc.shape[0]
    e = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_size(m, n, opts)
    if workspace is None:
        ws_keep, ws_ptr = _aligned_workspace(need, dev)
    else:
        ws_keep, ws_ptr = workspace, workspace.data_ptr()
        need = workspace.numel()
    rc = lib().trsyl_robust(m, n, Ac.data_ptr(), max(1, m), Bc.data_ptr(), max(1, n),
                            Yc.data_ptr(), max(1, m), e.data_ptr(), sc.data_ptr(), info.data_ptr(),
                            ctypes.byref(opts), ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_robust rejected its arguments: {rc}")
    solve_async._keep = (Ac, Bc, ws_keep)  # keep inputs alive until the caller synchronises
    return Yc, e, sc, info


def solve(A, B, C, **kw):
    """Robust solve; returns (Y (m x n, column-major view), e (alpha = 2^-e), info)."""
    Yc, e, sc, info = solve_async(A, B, C, make_opts(**kw))
    torch.cuda.synchronize(Yc.device)
    return Yc.t(), int(e.item()), int(info.item())


def debug_protect_update(args) -> list[int]:
    a = torch.as_tensor(args, dtype=torch.float64).reshape(-1).cuda()
    out = torch.zeros(a.numel() // 3, dtype=torch.int32, device=a.device)
    rc = lib().trsyl_debug_protect_update(out.numel(), a.data_ptr(), out.data_ptr(), _stream(a.device))
    if rc:
        raise RuntimeError(rc)
    return out.cpu().tolist()


def debug_protect_division(args) -> list[int]:
    a = torch.as_tensor(args, dtype=torch.float64).reshape(-1).cuda()
    out = torch.zeros(a.numel() // 2, dtype=torch.int32, device=a.device)
    rc = lib().trsyl_debug_protect_division(out.numel(), a.data_ptr(), out.data_ptr(), _stream(a.device))
    if rc:
        raise RuntimeError(rc)
    return out.cpu().tolist()
