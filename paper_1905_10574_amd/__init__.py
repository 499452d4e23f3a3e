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

__all__ = ["Opts", "lib", "solve", "solve_async", "adjoint", "adjoint_async", "grad", "residual", "trsyl",
           "solve_batched", "solve_batched_async", "autotune_tiles", "save_tile_table", "load_tile_table",
           "debug_protect_update", "debug_protect_division", "debug_task_order", "TrsylFunction", "workspace_size",
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
                ("trace", ctypes.c_void_p), ("counters", ctypes.c_void_p)]


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
        L.trsyl_robust_noalloc.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _P,
                                           ctypes.POINTER(Opts), _P]
        L.trsyl_robust_noalloc.restype = ctypes.c_int
        L.trsyl_adjoint_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(Opts)]
        L.trsyl_adjoint_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_adjoint.argtypes = L.trsyl_robust.argtypes
        L.trsyl_robust_adjoint.restype = ctypes.c_int
        L.trsyl_sync_result.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.trsyl_sync_result.restype = ctypes.c_int
        L.trsyl_general_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(Opts)]
        L.trsyl_general_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_general.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int32] + list(L.trsyl_robust.argtypes)
        L.trsyl_robust_general.restype = ctypes.c_int
        L.trsyl_bartels_stewart_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(Opts)]
        L.trsyl_bartels_stewart_workspace_size.restype = ctypes.c_size_t
        L.trsyl_bartels_stewart.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _I64,
                                            _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.trsyl_bartels_stewart.restype = ctypes.c_int
        L.trsyl_grad.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P,
                                 _P, _I64, _P, _I64, _P, _I64, _P]
        L.trsyl_grad.restype = ctypes.c_int
        L.trsyl_residual_workspace_size.argtypes = [_I64, _I64]
        L.trsyl_residual_workspace_size.restype = ctypes.c_size_t
        L.trsyl_residual.argtypes = [_I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P, _P,
                                     ctypes.c_size_t, _P]
        L.trsyl_residual.restype = ctypes.c_int
        L.trsyl_batched_workspace_size.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.POINTER(Opts)]
        L.trsyl_batched_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_batched.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                           ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P]
        L.trsyl_robust_batched.restype = ctypes.c_int
        L.trsyl_adjoint_batched_workspace_size.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.POINTER(Opts)]
        L.trsyl_adjoint_batched_workspace_size.restype = ctypes.c_size_t
        L.trsyl_robust_adjoint_batched.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                                   _P, ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P]
        L.trsyl_robust_adjoint_batched.restype = ctypes.c_int
        L.trsyl_debug_protect_update.argtypes = [ctypes.c_int32, _P, _P, _P]
        L.trsyl_debug_protect_update.restype = ctypes.c_int
        L.trsyl_debug_protect_division.argtypes = [ctypes.c_int32, _P, _P, _P]
        L.trsyl_debug_protect_division.restype = ctypes.c_int
        L.trsyl_debug_task_order.argtypes = [ctypes.c_int32] * 7 + [_P, _I64]
        L.trsyl_debug_task_order.restype = _I64
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


def colmajor(X: torch.Tensor, device=None, fresh: bool = False) -> torch.Tensor:
    """Column-major float64 copy on the device, returned as its transposed (row-major) storage
    tensor S with S.t() == X; S.data_ptr() is the column-major buffer with ld = X.shape[0].
    When X already is a column-major float64 tensor on that device, S shares X's storage; with
    fresh=True (operands the library overwrites) S is always a new buffer, so the caller's
    tensor is never written."""
    if not isinstance(X, torch.Tensor):
        X = torch.as_tensor(X)
    if device is None:
        device = X.device if X.is_cuda else torch.device("cuda")
    S = X.to(device=device, dtype=torch.float64).t().contiguous()
    if fresh and S.numel() > 0 and S.untyped_storage().data_ptr() == X.untyped_storage().data_ptr():
        S = S.clone()
    return S


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
    Yc = colmajor(C, dev, fresh=True)
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


NOALLOC_BYTES = 64 << 20      # TRSYL_NOALLOC_BYTES
ENOSPACE = -201               # TRSYL_ENOSPACE


def solve_noalloc_async(A, B, C, opts: Opts | None = None):
    """Enqueue trsyl_robust_noalloc (the solve that allocates nothing on the device: its state lives
    in the library's fixed per-GPU array) on the current stream.  Returns (Ys, e, scale, info) as
    solve_async does; raises on a rejected call (TRSYL_ENOSPACE for a problem too large for it)."""
    opts = opts or make_opts()
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Yc = colmajor(C, dev, fresh=True)
    m, n = Yc.shape[1], Yc.shape[0]
    e = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    rc = lib().trsyl_robust_noalloc(m, n, Ac.data_ptr(), max(1, m), Bc.data_ptr(), max(1, n), Yc.data_ptr(),
                                    max(1, m), e.data_ptr(), sc.data_ptr(), info.data_ptr(), ctypes.byref(opts),
                                    _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_robust_noalloc rejected the call: {rc}")
    solve_noalloc_async._keep = (Ac, Bc)
    return Yc, e, sc, info


def sync_result(e, scale, info, stream=None) -> tuple[int, float, int]:
    """(e, alpha, info) of a solve enqueued with solve_async, read back by trsyl_sync_result."""
    eh, sh, ih = ctypes.c_int64(0), ctypes.c_double(0.0), ctypes.c_int32(0)
    st = stream if stream is not None else _stream(e.device)
    rc = lib().trsyl_sync_result(e.data_ptr(), scale.data_ptr(), info.data_ptr(), ctypes.byref(eh),
                                 ctypes.byref(sh), ctypes.byref(ih), st)
    if rc != 0:
        raise RuntimeError(f"trsyl_sync_result failed: {rc}")
    return int(eh.value), float(sh.value), int(ih.value)


def solve(A, B, C, *, counters=False, **kw):
    """Robust solve; returns (Y (m x n, column-major view), e (alpha = 2^-e), info), and with
    counters=True also the scaling-event counts {"fallback_solves" (element-level Algorithm 2),
    "scaled_updates", "scaled_solves" (leaf-tiled robust tile solves), "refine_sweeps" (sweeps of
    the precision form that updated Y)}."""
    opts = make_opts(**kw)
    cnt = None
    if counters:
        dev = torch.device("cuda", torch.cuda.current_device())
        cnt = torch.zeros(4, dtype=torch.int32, device=dev)
        opts.counters = cnt.data_ptr()
    Yc, e, sc, info = solve_async(A, B, C, opts)
    torch.cuda.synchronize(Yc.device)
    out = (Yc.t(), int(e.item()), int(info.item()))
    if counters:
        c = cnt.cpu().tolist()
        out = out + ({"fallback_solves": c[0], "scaled_updates": c[1], "scaled_solves": c[2],
                      "refine_sweeps": c[3]},)
    return out


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


FLAG_ROBUST_SOLVE, FLAG_PAIRED_UPDATES, FLAG_DEFERRED_UPDATES = 1, 4, 8


def debug_task_order(pt: int, qt: int, tile_m: int = 128, tile_n: int = 0, slabs: int = 1,
                     workers: int = 256, flags: int = 0):
    """The persistent scheduler's static task order for a pt x qt tile grid (host only), as a
    numpy uint64 array of task words (see trsyl_debug_task_order)."""
    import numpy as np
    args = (int(pt), int(qt), int(tile_m), int(tile_n or tile_m), int(slabs), int(workers), int(flags))
    n = lib().trsyl_debug_task_order(*args, None, 0)
    if n < 0:
        raise ValueError(f"trsyl_debug_task_order: {n}")
    out = np.zeros(max(int(n), 1), dtype=np.uint64)
    n2 = lib().trsyl_debug_task_order(*args, out.ctypes.data, int(n))
    if n2 != n:
        raise RuntimeError(f"trsyl_debug_task_order: {n2}")
    return out[:n]


def adjoint_async(A, B, W, opts: Opts | None = None):
    """Enqueue the adjoint solve A^T G + G B^T = alpha_G W.  Returns (Gs, eG, info) device tensors
    with Gs the column-major storage of G (G = Gs.t())."""
    opts = opts or make_opts()
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Gc = colmajor(W, dev, fresh=True)
    m, n = Gc.shape[1], Gc.shape[0]
    e = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = int(lib().trsyl_adjoint_workspace_size(m, n, ctypes.byref(opts)))
    ws_keep, ws_ptr = _aligned_workspace(need, dev)
    rc = lib().trsyl_robust_adjoint(m, n, Ac.data_ptr(), max(1, m), Bc.data_ptr(), max(1, n),
                                    Gc.data_ptr(), max(1, m), e.data_ptr(), sc.data_ptr(),
                                    info.data_ptr(), ctypes.byref(opts), ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_robust_adjoint rejected its arguments: {rc}")
    adjoint_async._keep = (Ac, Bc, ws_keep)
    return Gc, e, info


def adjoint(A, B, W, **kw):
    """Adjoint solve; returns (G, eG, info) with A^T G + G B^T = 2^-eG W."""
    Gc, e, info = adjoint_async(A, B, W, make_opts(**kw))
    torch.cuda.synchronize(Gc.device)
    return Gc.t(), int(e.item()), int(info.item())


def general_async(A, B, C, trana="N", tranb="N", isgn=1, opts: Opts | None = None):
    """Enqueue op(A) Y + isgn Y op(B) = alpha C (op(X) = X for "N", X^T for "T").  Returns
    (Ys, e, info) device tensors with Ys the column-major storage of Y (Y = Ys.t())."""
    opts = opts or make_opts()
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Yc = colmajor(C, dev, fresh=True)
    m, n = Yc.shape[1], Yc.shape[0]
    e = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = int(lib().trsyl_general_workspace_size(m, n, ctypes.byref(opts)))
    ws_keep, ws_ptr = _aligned_workspace(need, dev)
    rc = lib().trsyl_robust_general(trana.encode(), tranb.encode(), int(isgn), m, n, Ac.data_ptr(),
                                    max(1, m), Bc.data_ptr(), max(1, n), Yc.data_ptr(), max(1, m),
                                    e.data_ptr(), sc.data_ptr(), info.data_ptr(), ctypes.byref(opts),
                                    ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_robust_general rejected its arguments: {rc}")
    general_async._keep = (Ac, Bc, ws_keep)
    return Yc, e, info


def solve_general(A, B, C, trana="N", tranb="N", isgn=1, **kw):
    """General-form solve; returns (Y, e, info) with op(A) Y + isgn Y op(B) = 2^-e C."""
    Yc, e, info = general_async(A, B, C, trana, tranb, isgn, make_opts(**kw))
    torch.cuda.synchronize(Yc.device)
    return Yc.t(), int(e.item()), int(info.item())


def lyapunov(A, C, **kw):
    """Lyapunov solve A Y + Y A^T = 2^-e C (A upper quasi-triangular); returns (Y, e, info)."""
    return solve_general(A, A, C, "N", "T", 1, **kw)


def bartels_stewart(U, At, V, Bt, C, **kw):
    """A X + X B = 2^-e C from the real Schur forms A = U At U^T, B = V Bt V^T (computed by the
    caller); returns (X, e, info)."""
    opts = make_opts(**kw)
    Uc = colmajor(U)
    dev = Uc.device
    Atc, Vc, Btc, Xc = colmajor(At, dev), colmajor(V, dev), colmajor(Bt, dev), colmajor(C, dev, fresh=True)
    m, n = Xc.shape[1], Xc.shape[0]
    e = torch.zeros(1, dtype=torch.int64, device=dev)
    sc = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    need = int(lib().trsyl_bartels_stewart_workspace_size(m, n, ctypes.byref(opts)))
    ws_keep, ws_ptr = _aligned_workspace(need, dev)
    rc = lib().trsyl_bartels_stewart(m, n, Uc.data_ptr(), max(1, m), Atc.data_ptr(), max(1, m),
                                     Vc.data_ptr(), max(1, n), Btc.data_ptr(), max(1, n), Xc.data_ptr(),
                                     max(1, m), e.data_ptr(), sc.data_ptr(), info.data_ptr(),
                                     ctypes.byref(opts), ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_bartels_stewart rejected its arguments: {rc}")
    torch.cuda.synchronize(dev)
    del ws_keep
    return Xc.t(), int(e.item()), int(info.item())


def grad(A, B, Y, eY, G, eG):
    """Gradient products for L = <W, Y> (Y the scaled forward output, alpha_Y = 2^-eY fixed) from the
    adjoint output G (A^T G + G B^T = 2^-eG W): returns (dA, dB, dC) on the device, dA and dB
    masked to the quasi-triangular patterns of A and B.  eY, eG: ints or int64 device tensors."""
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Yc = colmajor(Y, dev)
    Gc = colmajor(G, dev)
    m, n = Yc.shape[1], Yc.shape[0]
    eYt = eY if isinstance(eY, torch.Tensor) else torch.tensor([int(eY)], dtype=torch.int64, device=dev)
    eGt = eG if isinstance(eG, torch.Tensor) else torch.tensor([int(eG)], dtype=torch.int64, device=dev)
    dA = torch.empty(m, m, dtype=torch.float64, device=dev)    # column-major storage
    dB = torch.empty(n, n, dtype=torch.float64, device=dev)
    dC = torch.empty(n, m, dtype=torch.float64, device=dev)
    rc = lib().trsyl_grad(m, n, Ac.data_ptr(), max(1, m), Bc.data_ptr(), max(1, n), Yc.data_ptr(),
                          max(1, m), eYt.data_ptr(), Gc.data_ptr(), max(1, m), eGt.data_ptr(),
                          dA.data_ptr(), max(1, m), dB.data_ptr(), max(1, n), dC.data_ptr(),
                          max(1, m), _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_grad rejected its arguments: {rc}")
    grad._keep = (Ac, Bc, Yc, Gc, eYt, eGt)
    return dA.t(), dB.t(), dC.t()


def residual(A, B, Y, e, C) -> float:
    """Eq. (9) relative residual of (alpha = 2^-e, Y), evaluated on the device in FP64."""
    Ac = colmajor(A)
    dev = Ac.device
    Bc = colmajor(B, dev)
    Yc = colmajor(Y, dev)
    Cc = colmajor(C, dev)
    m, n = Yc.shape[1], Yc.shape[0]
    et = e if isinstance(e, torch.Tensor) else torch.tensor([int(e)], dtype=torch.int64, device=dev)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    need = int(lib().trsyl_residual_workspace_size(m, n))
    ws_keep, ws_ptr = _aligned_workspace(need, dev)
    rc = lib().trsyl_residual(m, n, Ac.data_ptr(), max(1, m), Bc.data_ptr(), max(1, n), Yc.data_ptr(),
                              max(1, m), et.data_ptr(), Cc.data_ptr(), max(1, m), out.data_ptr(),
                              ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"trsyl_residual rejected its arguments: {rc}")
    torch.cuda.synchronize(dev)
    del ws_keep
    return float(out.item())


class TrsylFunction(torch.autograd.Function):
    """Y = trsyl(A, B, C): the robust solution of A Y + Y B = alpha C with alpha = 2^-e held fixed
    (e is returned as a non-differentiable output).  The backward pass solves the adjoint
    A^T G + G B^T = alpha_G dL/dY on the device and forms dA = -G~ Y^T (A's pattern),
    dB = -Y^T G~ (B's pattern), dC = alpha G~ with G~ = G / alpha_G."""

    @staticmethod
    def forward(ctx, A, B, C, tile=None):
        Yc, e, _, info = solve_async(A, B, C, make_opts(tile=tile))
        torch.cuda.synchronize(Yc.device)
        Y = Yc.t().contiguous()
        ctx.save_for_backward(A, B, Y, e)
        ctx.tile = tile
        ctx.mark_non_differentiable(e)
        ctx.c_dtype = C.dtype if isinstance(C, torch.Tensor) else torch.float64
        return Y, e

    @staticmethod
    def backward(ctx, dY, de):
        A, B, Y, e = ctx.saved_tensors
        G, eG, info = adjoint(A, B, dY.to(torch.float64), tile=ctx.tile)
        dA, dB, dC = grad(A, B, Y, e, G, eG)
        torch.cuda.synchronize(Y.device)
        return dA.to(A.dtype), dB.to(B.dtype), dC.to(ctx.c_dtype), None


def trsyl(A, B, C, tile=None):
    """Differentiable robust solve: returns (Y, e) with A Y + Y B = 2^-e C."""
    return TrsylFunction.apply(A, B, C, tile)


def _batched_async(As, Bs, Cs, tiles, opts, adjoint):
    opts = opts or make_opts()
    count = len(As)
    Acs = [colmajor(A) for A in As]
    dev = Acs[0].device if count else torch.device("cuda")
    Bcs = [colmajor(B, dev) for B in Bs]
    Ycs = [colmajor(C, dev, fresh=True) for C in Cs]
    ms = [Y.shape[1] for Y in Ycs]
    ns = [Y.shape[0] for Y in Ycs]
    if isinstance(tiles, str) and tiles == "auto":
        tiles = [(tile_for(mi), tile_for(ni)) for mi, ni in zip(ms, ns)]
    I64 = ctypes.c_int64 * count
    m_a, n_a = I64(*ms), I64(*ns)
    lda, ldb = I64(*[max(1, x) for x in ms]), I64(*[max(1, x) for x in ns])
    ldc = I64(*[max(1, x) for x in ms])
    Pa = ctypes.c_void_p * count
    A_p, B_p, C_p = Pa(*[a.data_ptr() for a in Acs]), Pa(*[b.data_ptr() for b in Bcs]), Pa(*[y.data_ptr() for y in Ycs])
    t_a = None
    if tiles is not None:
        t_a = (ctypes.c_int32 * (2 * count))(*[int(v) for tt in tiles for v in tt])
    e = torch.zeros(max(count, 1), dtype=torch.int64, device=dev)
    sc = torch.zeros(max(count, 1), dtype=torch.float64, device=dev)
    info = torch.zeros(max(count, 1), dtype=torch.int32, device=dev)
    L = lib()
    size_fn = L.trsyl_adjoint_batched_workspace_size if adjoint else L.trsyl_batched_workspace_size
    entry = L.trsyl_robust_adjoint_batched if adjoint else L.trsyl_robust_batched
    need = int(size_fn(count, m_a, n_a, t_a, ctypes.byref(opts)))
    if need == 0 and count > 0:
        raise RuntimeError("the batched workspace query rejected the arguments")
    ws_keep, ws_ptr = _aligned_workspace(max(need, 256), dev)
    rc = entry(count, m_a, n_a, A_p, lda, B_p, ldb, C_p, ldc, t_a, e.data_ptr(), sc.data_ptr(),
               info.data_ptr(), ctypes.byref(opts), ws_ptr, need, _stream(dev))
    if rc != 0:
        raise RuntimeError(f"the batched solve rejected its arguments: {rc}")
    _batched_async._keep = (Acs, Bcs, ws_keep, m_a, n_a, A_p, B_p, C_p, t_a)
    return Ycs, e, info


def solve_batched_async(As, Bs, Cs, tiles=None, opts: Opts | None = None):
    """Enqueue one batched robust solve of len(As) independent problems on the current stream.
    tiles: None (opts' tile for all), "auto" (the autotuner's table), or a list of (tile_m, tile_n).
    Returns (Ys, e, info): Ys the column-major storages (Y_i = Ys[i].t()), e / info device tensors."""
    return _batched_async(As, Bs, Cs, tiles, opts, False)


def adjoint_batched_async(As, Bs, Ws, tiles=None, opts: Opts | None = None):
    """Enqueue one batched adjoint solve A_i^T G_i + G_i B_i^T = 2^-e_i W_i; returns (Gs, e, info)
    as solve_batched_async does."""
    return _batched_async(As, Bs, Ws, tiles, opts, True)


def adjoint_batched(As, Bs, Ws, tiles=None, **kw):
    """Batched adjoint solve; returns a list of (G, eG, info)."""
    Gcs, e, info = adjoint_batched_async(As, Bs, Ws, tiles, make_opts(**kw))
    if Gcs:
        torch.cuda.synchronize(Gcs[0].device)
    es, infos = e.cpu().tolist(), info.cpu().tolist()
    return [(G.t(), int(es[i]), int(infos[i])) for i, G in enumerate(Gcs)]


def solve_batched(As, Bs, Cs, tiles=None, **kw):
    """Batched robust solve; returns a list of (Y, e, info)."""
    Ycs, e, info = solve_batched_async(As, Bs, Cs, tiles, make_opts(**kw))
    if Ycs:
        torch.cuda.synchronize(Ycs[0].device)
    es, infos = e.cpu().tolist(), info.cpu().tolist()
    return [(Y.t(), es[i], infos[i]) for i, Y in enumerate(Ycs)]


# ---------------------------------------------------------------------------------------------
# Tile autotuner for batched solves.  For each size bucket (powers of two), a batch of synthetic
# problems of that size is solved with every candidate tile: half separated (upper triangular,
# diagonal U[1,10], strictly upper N(0,1)/sqrt(n), C N(0,1)) and half growth (diagonals of A and
# -B within [1e-3, 1e-2] of each other, strictly upper U[-10,10], C U[-1,1]), the two kinds of the
# batched workload.  Following the paper's tuning protocol (Sec. 3), each candidate is timed three
# times after one warm-up run and ranked by its median; the tile with the best median wins.  The
# inputs are staged once, outside the timed region.  The table can be saved to and loaded from a
# JSON file (bucket -> tile).
# ---------------------------------------------------------------------------------------------
_TILE_TABLE: dict[int, int] = {}
TILE_CANDIDATES = (16, 32, 48, 64, 96, 128)
BUCKETS = (64, 128, 256, 512, 1024, 2048)


def tile_for(x: int) -> int:
    """Autotuned tile for a dimension of size x: the entry of the nearest tuned bucket (by ratio);
    before a table is tuned or loaded, 128 (or x itself for small x, at least 16)."""
    if not _TILE_TABLE:
        return 128 if x >= 128 else max(16, min(128, x))
    import math
    lx = math.log(max(1, x))
    b = min(_TILE_TABLE, key=lambda k: (abs(math.log(k) - lx), k))
    return _TILE_TABLE[b]


def save_tile_table(path: str, meta: dict | None = None) -> None:
    """Write the current table as JSON: {"tiles": {bucket: tile}, "meta": {...}}."""
    import json
    with open(path, "w") as fh:
        json.dump({"tiles": {str(k): int(v) for k, v in sorted(_TILE_TABLE.items())}, "meta": meta or {}},
                  fh, indent=1)


def load_tile_table(path: str) -> dict[int, int]:
    """Replace the current table by the one in a JSON file written by save_tile_table."""
    import json
    with open(path) as fh:
        rec = json.load(fh)
    tiles = {int(k): int(v) for k, v in rec["tiles"].items()}
    if not tiles or any(b <= 0 or t <= 0 for b, t in tiles.items()):
        raise ValueError(f"{path}: not a tile table")
    _TILE_TABLE.clear()
    _TILE_TABLE.update(tiles)
    return dict(_TILE_TABLE)


def _tuning_problem(gen, s: int, growth: bool):
    """One synthetic tuning problem of order s (torch CPU tensors, float64)."""
    if not growth:
        A = torch.triu(torch.randn(s, s, generator=gen, dtype=torch.float64), 1) / s ** 0.5
        A += torch.diag(torch.rand(s, generator=gen, dtype=torch.float64) * 9 + 1)
        B = torch.triu(torch.randn(s, s, generator=gen, dtype=torch.float64), 1) / s ** 0.5
        B += torch.diag(torch.rand(s, generator=gen, dtype=torch.float64) * 9 + 1)
        C = torch.randn(s, s, generator=gen, dtype=torch.float64)
        return A, B, C
    la = (torch.rand(s, generator=gen, dtype=torch.float64) * 2 - 1) * 1e-2
    u = torch.rand(s, generator=gen, dtype=torch.float64) * 9e-3 + 1e-3
    sg = torch.where(torch.rand(s, generator=gen) < 0.5, 1.0, -1.0).to(torch.float64)
    lb = -la + sg * u
    A = torch.triu((torch.rand(s, s, generator=gen, dtype=torch.float64) * 2 - 1) * 10, 1) + torch.diag(la)
    B = torch.triu((torch.rand(s, s, generator=gen, dtype=torch.float64) * 2 - 1) * 10, 1) + torch.diag(lb)
    C = torch.rand(s, s, generator=gen, dtype=torch.float64) * 2 - 1
    return A, B, C


def autotune_tiles(buckets=BUCKETS, candidates=TILE_CANDIDATES, batch_flops=2e10, reps=3, seed=0,
                   device=None, path: str | None = None) -> dict[int, int]:
    """Measure and store the best tile per size bucket (best median of `reps` timed runs after
    one warm-up run); returns the table, and writes it to `path` as JSON when given."""
    import statistics
    device = device or torch.device("cuda")
    gen = torch.Generator(device="cpu").manual_seed(seed)
    medians = {}
    for s in buckets:
        count = int(max(2, min(64, batch_flops // (2.0 * s ** 3))))
        probs = [_tuning_problem(gen, s, growth=(i % 2 == 1)) for i in range(count)]
        As = [p[0].to(device) for p in probs]
        Bs = [p[1].to(device) for p in probs]
        Cs = [p[2].to(device) for p in probs]
        best, best_t = None, None
        for t in candidates:
            if t > max(16, s):
                continue
            opts = make_opts(tile=t)
            times = []
            for _ in range(reps + 1):
                torch.cuda.synchronize(device)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record()
                solve_batched_async(As, Bs, Cs, [(t, t)] * count, opts)
                ev1.record()
                torch.cuda.synchronize(device)
                times.append(ev0.elapsed_time(ev1))
            tm = statistics.median(times[1:])
            medians.setdefault(s, {})[t] = tm
            if best is None or tm < best:
                best, best_t = tm, t
        _TILE_TABLE[s] = best_t
    if path:
        save_tile_table(path, {"protocol": f"best median of {reps} timed runs after 1 warm-up",
                               "batch_flops": batch_flops, "candidates": list(candidates),
                               "median_ms": {str(k): {str(t): round(v, 4) for t, v in m.items()}
                                             for k, m in medians.items()},
                               "device": torch.cuda.get_device_name(device)})
    return dict(_TILE_TABLE)
