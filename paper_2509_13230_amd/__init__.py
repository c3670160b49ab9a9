"""MI355X sampler for the maximum-entropy configuration models (UBCM / UECM).

Thin Python binding over the C-ABI of ``libmh.so`` (declared in
``include/mh.h``).  PyTorch provides device memory and the current HIP
stream; every step of the sampling path runs in the library's HIP kernels.
There is no CPU fallback: without the built library every call raises.

    import torch, paper_2509_13230_amd as mh
    x = torch.rand(1000, dtype=torch.float64, device="cuda") * 0.1
    src, dst = mh.sample_unweighted(x, seed=1)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "MHError", "lib", "library_path",
    "sample_unweighted", "sample_weighted", "sample_bruteforce",
    "order", "bound", "plan_counts",
    "expected_degree", "expected_degree_grad", "ExpectedDegree",
    "Stats", "DEFAULT_SEG_WORK",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmh.so")

DEFAULT_SEG_WORK = 32

MH_OK, MH_EINVAL, MH_ECAPACITY, MH_EHIP, MH_EWORKSPACE = 0, -1, -2, -3, -4


class MHError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_status_text(status)} (status {status})")


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("steps", "proposals", "accepts", "segments", "saturated_w", "n_edges")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class PlanParams(ctypes.Structure):
    _fields_ = [("seg_work", ctypes.c_int32), ("flags", ctypes.c_uint32), ("stage_events", ctypes.c_void_p)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load libmh.so (built in-tree by ``python -m paper_2509_13230_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run `python -m paper_2509_13230_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, u32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_size_t)
    P = ctypes.POINTER
    sig = {
        "mh_workspace_bytes": ([i64, ctypes.c_int, P(PlanParams)], sz),
        "mh_sample_unweighted": ([vp, i64, u64, u32, P(PlanParams), vp, vp, i64, P(i64), vp, sz, P(Stats), vp], ctypes.c_int),
        "mh_sample_weighted": ([vp, vp, i64, u64, u32, P(PlanParams), vp, vp, vp, i64, P(i64), vp, sz, P(Stats), vp],
                               ctypes.c_int),
        "mh_bruteforce_workspace_bytes": ([i64], sz),
        "mh_sample_bruteforce": ([vp, vp, i64, u64, u32, i64, i64, vp, vp, vp, i64, P(i64), vp, sz, vp], ctypes.c_int),
        "mh_order": ([vp, vp, i64, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "mh_bound_workspace_bytes": ([i64], sz),
        "mh_bound": ([vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "mh_plan_workspace_bytes": ([i64], sz),
        "mh_plan_counts": ([vp, vp, i64, i32, vp, vp, sz, vp], ctypes.c_int),
        "mh_expected_degree_fwd": ([vp, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "mh_expected_degree_bwd": ([vp, vp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "mh_status_string": ([ctypes.c_int], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _status_text(status: int) -> str:
    try:
        return lib().mh_status_string(status).decode()
    except Exception:
        return "unknown"


def _check(status: int, what: str):
    if status != MH_OK:
        raise MHError(status, what)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return t.contiguous()


def _workspace(nbytes: int, device: torch.device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class SampleResult:
    src: torch.Tensor
    dst: torch.Tensor
    w: torch.Tensor | None
    stats: dict | None


def _sample(x, y, seed, replica, seg_work, capacity, stats, out, workspace, stage_events=None):
    x = _dev_f64(x, "x")
    if y is not None:
        y = _dev_f64(y, "y")
        if y.shape != x.shape:
            raise ValueError("x and y must have the same shape")
    n = x.numel()
    dev = x.device
    L = lib()
    plan = PlanParams(int(seg_work), 0, stage_events)
    wsb = L.mh_workspace_bytes(n, 1 if y is not None else 0, ctypes.byref(plan))
    ws = workspace if workspace is not None and workspace.numel() >= wsb else _workspace(wsb, dev)
    cap = int(capacity) if capacity is not None else max(4096, 4 * n)
    if out is not None:
        src, dst = out[0], out[1]
        w = out[2] if y is not None else None
        cap = min(src.numel(), dst.numel(), w.numel() if w is not None else src.numel())
    else:
        src = dst = w = None
    nedge = ctypes.c_int64(0)
    st = Stats()
    for _attempt in range(2):
        if src is None or src.numel() < cap:
            src = torch.empty(cap, dtype=torch.int32, device=dev)
            dst = torch.empty(cap, dtype=torch.int32, device=dev)
            w = torch.empty(cap, dtype=torch.int32, device=dev) if y is not None else None
        sp = ctypes.byref(st) if stats else None
        if y is None:
            status = L.mh_sample_unweighted(_ptr(x), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst), cap,
                                            ctypes.byref(nedge), _ptr(ws), ws.numel(), sp, _stream(dev))
        else:
            status = L.mh_sample_weighted(_ptr(x), _ptr(y), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst),
                                          _ptr(w), cap, ctypes.byref(nedge), _ptr(ws), ws.numel(), sp, _stream(dev))
        if status == MH_ECAPACITY and out is None:
            cap = int(nedge.value)
            src = None
            continue
        _check(status, "mh_sample_weighted" if y is not None else "mh_sample_unweighted")
        break
    m = int(nedge.value)
    return SampleResult(src[:m], dst[:m], None if w is None else w[:m], st.as_dict() if stats else None)


def sample_unweighted(x: torch.Tensor, seed: int = 1, replica: int = 0, seg_work: int = DEFAULT_SEG_WORK,
                      capacity: int | None = None, stats: bool = False, out=None, workspace=None,
                      stage_events=None):
    """One sample of the unweighted model (Sec. 2.4).  Returns (src, dst) int32
    tensors, plus a stats dict when stats=True.  ``out=(src, dst)`` reuses
    buffers (then MH_ECAPACITY raises instead of retrying).  ``stage_events``:
    address of an array of 4 hipEvent_t recorded at the stage boundaries."""
    r = _sample(x, None, seed, replica, seg_work, capacity, stats, out, workspace, stage_events)
    return (r.src, r.dst, r.stats) if stats else (r.src, r.dst)


def sample_weighted(x: torch.Tensor, y: torch.Tensor, seed: int = 1, replica: int = 0,
                    seg_work: int = DEFAULT_SEG_WORK, capacity: int | None = None, stats: bool = False, out=None,
                    workspace=None, stage_events=None):
    """One sample of the weighted model (Sec. 2.5, Alg. 1): (src, dst, w)."""
    r = _sample(x, y, seed, replica, seg_work, capacity, stats, out, workspace, stage_events)
    return (r.src, r.dst, r.w, r.stats) if stats else (r.src, r.dst, r.w)


def sample_bruteforce(x: torch.Tensor, y: torch.Tensor | None = None, seed: int = 1, replica: int = 0,
                      row_begin: int = 0, row_end: int | None = None, capacity: int | None = None, out=None):
    """Brute-force sampler over all pairs (Sec. 2.2): (src, dst[, w]) with src < dst."""
    x = _dev_f64(x, "x")
    if y is not None:
        y = _dev_f64(y, "y")
    n = x.numel()
    dev = x.device
    L = lib()
    re = n if row_end is None else int(row_end)
    ws = _workspace(L.mh_bruteforce_workspace_bytes(n), dev)
    cap = int(capacity) if capacity is not None else max(4096, 4 * n)
    src = dst = w = None
    if out is not None:
        src, dst = out[0], out[1]
        w = out[2] if y is not None else None
        cap = src.numel()
    nedge = ctypes.c_int64(0)
    for _attempt in range(2):
        if src is None:
            src = torch.empty(cap, dtype=torch.int32, device=dev)
            dst = torch.empty(cap, dtype=torch.int32, device=dev)
            w = torch.empty(cap, dtype=torch.int32, device=dev) if y is not None else None
        status = L.mh_sample_bruteforce(_ptr(x), _ptr(y), n, seed, replica, int(row_begin), re, _ptr(src), _ptr(dst),
                                        _ptr(w), cap, ctypes.byref(nedge), _ptr(ws), ws.numel(), _stream(dev))
        if status == MH_ECAPACITY and out is None:
            cap = int(nedge.value)
            src = None
            continue
        _check(status, "mh_sample_bruteforce")
        break
    m = int(nedge.value)
    return (src[:m], dst[:m]) if y is None else (src[:m], dst[:m], w[:m])


def order(x: torch.Tensor, y: torch.Tensor | None = None):
    """Node order (descending x, or x*y; ties by id): (perm, zs, ys|None, status).
    status is a device int32 tensor: nonzero when the parameters are invalid."""
    x = _dev_f64(x, "x")
    y = None if y is None else _dev_f64(y, "y")
    n = x.numel()
    dev = x.device
    L = lib()
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    zs = torch.empty(n, dtype=torch.float64, device=dev)
    ys = torch.empty(n, dtype=torch.float64, device=dev) if y is not None else None
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    plan = PlanParams(DEFAULT_SEG_WORK, 0, None)
    ws = _workspace(L.mh_workspace_bytes(n, 1 if y is not None else 0, ctypes.byref(plan)), dev)
    _check(L.mh_order(_ptr(x), _ptr(y), n, _ptr(perm), _ptr(zs), _ptr(ys), _ptr(status), _ptr(ws), ws.numel(),
                      _stream(dev)), "mh_order")
    return perm, zs, ys, status


def bound(ys: torch.Tensor) -> torch.Tensor:
    """c[r] = 1 - (product of the two largest ys over ranks r..n-1)."""
    ys = _dev_f64(ys, "ys")
    n = ys.numel()
    L = lib()
    c = torch.empty(n, dtype=torch.float64, device=ys.device)
    ws = _workspace(L.mh_bound_workspace_bytes(n), ys.device)
    _check(L.mh_bound(_ptr(ys), n, _ptr(c), _ptr(ws), ws.numel(), _stream(ys.device)), "mh_bound")
    return c


def plan_counts(zs: torch.Tensor, c: torch.Tensor | None, seg_work: int = DEFAULT_SEG_WORK) -> torch.Tensor:
    """Segments per row of the sweep plan."""
    zs = _dev_f64(zs, "zs")
    c = None if c is None else _dev_f64(c, "c")
    n = zs.numel()
    L = lib()
    nseg = torch.empty(n, dtype=torch.int32, device=zs.device)
    ws = _workspace(L.mh_plan_workspace_bytes(n), zs.device)
    _check(L.mh_plan_counts(_ptr(zs), _ptr(c), n, int(seg_work), _ptr(nseg), _ptr(ws), ws.numel(),
                            _stream(zs.device)), "mh_plan_counts")
    return nseg


def expected_degree(x: torch.Tensor, y: torch.Tensor | None = None, mult: torch.Tensor | None = None):
    """(k, s): expected degrees (and strengths when y is given)."""
    x = _dev_f64(x, "x")
    y = None if y is None else _dev_f64(y, "y")
    mult = None if mult is None else _dev_f64(mult, "mult")
    n = x.numel()
    k = torch.empty(n, dtype=torch.float64, device=x.device)
    s = torch.empty(n, dtype=torch.float64, device=x.device) if y is not None else None
    _check(lib().mh_expected_degree_fwd(_ptr(x), _ptr(y), _ptr(mult), n, _ptr(k), _ptr(s), _stream(x.device)),
           "mh_expected_degree_fwd")
    return k, s


def expected_degree_grad(x, y, mult, gk, gs):
    """Adjoint of expected_degree: (gx, gy) for upstream (gk, gs)."""
    x = _dev_f64(x, "x")
    y = None if y is None else _dev_f64(y, "y")
    mult = None if mult is None else _dev_f64(mult, "mult")
    gk = _dev_f64(gk, "gk")
    gs = None if gs is None else _dev_f64(gs, "gs")
    if y is not None and gs is None:
        gs = torch.zeros_like(gk)
    n = x.numel()
    gx = torch.empty(n, dtype=torch.float64, device=x.device)
    gy = torch.empty(n, dtype=torch.float64, device=x.device) if y is not None else None
    _check(lib().mh_expected_degree_bwd(_ptr(x), _ptr(y), _ptr(mult), n, _ptr(gk), _ptr(gs), _ptr(gx), _ptr(gy),
                                        _stream(x.device)), "mh_expected_degree_bwd")
    return gx, gy


class ExpectedDegree(torch.autograd.Function):
    """Differentiable (k, s) = expected_degree(x, y, mult) with the hand-written adjoint kernel.

    Unweighted when y is None (then s is returned as an empty tensor)."""

    @staticmethod
    def forward(ctx, x, y=None, mult=None):
        k, s = expected_degree(x, y, mult)
        ctx.save_for_backward(x, y if y is not None else torch.empty(0, dtype=x.dtype, device=x.device),
                              mult if mult is not None else torch.empty(0, dtype=x.dtype, device=x.device))
        ctx.weighted = y is not None
        ctx.has_mult = mult is not None
        if s is None:
            s = torch.empty(0, dtype=x.dtype, device=x.device)
        return k, s

    @staticmethod
    def backward(ctx, gk, gs):
        x, y, mult = ctx.saved_tensors
        y = y if ctx.weighted else None
        mult = mult if ctx.has_mult else None
        if gk is None:
            gk = torch.zeros_like(x)
        if ctx.weighted and (gs is None or gs.numel() == 0):
            gs = torch.zeros_like(x)
        gx, gy = expected_degree_grad(x, y, mult, gk.contiguous(), gs.contiguous() if ctx.weighted else None)
        return gx, (gy if ctx.weighted else None), None
