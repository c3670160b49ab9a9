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

DEFAULT_SEG_WORK = 8

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
    _fields_ = [("seg_work", ctypes.c_int32), ("flags", ctypes.c_uint32), ("grid_blocks", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("stage_events", ctypes.c_void_p)]


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
        "mh_sample_unweighted_async": ([vp, i64, u64, u32, P(PlanParams), vp, vp, i64, vp, sz, vp], ctypes.c_int),
        "mh_sample_weighted_async": ([vp, vp, i64, u64, u32, P(PlanParams), vp, vp, vp, i64, vp, sz, vp],
                                     ctypes.c_int),
        "mh_sample_result": ([vp, sz, i64, P(i64), vp], ctypes.c_int),
        "mh_sample_unweighted_noalloc": ([vp, i64, u64, u32, P(PlanParams), vp, vp, i64, P(i64), P(Stats), vp],
                                         ctypes.c_int),
        "mh_bipartite_workspace_bytes": ([i64, i64, ctypes.c_int, P(PlanParams)], sz),
        "mh_sample_bipartite": ([vp, vp, i64, vp, vp, i64, u32, u64, u32, P(PlanParams), vp, vp, vp, i64, P(i64), vp,
                                 sz, P(Stats), vp], ctypes.c_int),
        "mh_bruteforce_workspace_bytes": ([i64], sz),
        "mh_sample_bruteforce": ([vp, vp, i64, u64, u32, i64, i64, vp, vp, vp, i64, P(i64), vp, sz, vp], ctypes.c_int),
        "mh_order": ([vp, vp, i64, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "mh_bound_workspace_bytes": ([i64], sz),
        "mh_bound": ([vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "mh_plan_workspace_bytes": ([i64], sz),
        "mh_plan_counts": ([vp, vp, i64, i32, vp, vp, sz, vp], ctypes.c_int),
        "mh_expected_degree_fwd": ([vp, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "mh_expected_degree_bwd": ([vp, vp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "mh_sort_edges_workspace_bytes": ([i64], sz),
        "mh_sort_edges": ([vp, vp, vp, i64, vp, sz, vp], ctypes.c_int),
        "mh_sample_chung_lu": ([vp, i64, u64, u32, P(PlanParams), vp, vp, i64, P(i64), vp, sz, P(Stats), vp],
                               ctypes.c_int),
        "mh_sample_rank_counts": ([vp, i64, i32, u64, u32, P(PlanParams), vp, P(i64), vp, sz, P(Stats), vp],
                                  ctypes.c_int),
        "mh_triangles_workspace_bytes": ([i64, i64], sz),
        "mh_count_triangles": ([vp, vp, i64, i64, P(u64), vp, sz, vp], ctypes.c_int),
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


MH_MODEL_UBCM = 0
MH_MODEL_CHUNG_LU = 1


def _sample(x, y, seed, replica, seg_work, capacity, stats, out, workspace, stage_events=None, grid_blocks=0,
            chung_lu=False):
    x = _dev_f64(x, "x")
    if y is not None:
        y = _dev_f64(y, "y")
        if y.shape != x.shape:
            raise ValueError("x and y must have the same shape")
    n = x.numel()
    dev = x.device
    L = lib()
    plan = PlanParams(int(seg_work), 0, int(grid_blocks), 0, stage_events)
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
        if chung_lu:
            status = L.mh_sample_chung_lu(_ptr(x), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst), cap,
                                          ctypes.byref(nedge), _ptr(ws), ws.numel(), sp, _stream(dev))
        elif y is None:
            status = L.mh_sample_unweighted(_ptr(x), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst), cap,
                                            ctypes.byref(nedge), _ptr(ws), ws.numel(), sp, _stream(dev))
        else:
            status = L.mh_sample_weighted(_ptr(x), _ptr(y), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst),
                                          _ptr(w), cap, ctypes.byref(nedge), _ptr(ws), ws.numel(), sp, _stream(dev))
        if status == MH_ECAPACITY and out is None:
            cap = int(nedge.value)
            src = None
            continue
        _check(status, "mh_sample_chung_lu" if chung_lu else
               "mh_sample_weighted" if y is not None else "mh_sample_unweighted")
        break
    m = int(nedge.value)
    return SampleResult(src[:m], dst[:m], None if w is None else w[:m], st.as_dict() if stats else None)


def sample_unweighted(x: torch.Tensor, seed: int = 1, replica: int = 0, seg_work: int = DEFAULT_SEG_WORK,
                      capacity: int | None = None, stats: bool = False, out=None, workspace=None,
                      stage_events=None, grid_blocks: int = 0):
    """One sample of the unweighted model (Sec. 2.4).  Returns (src, dst) int32
    tensors, plus a stats dict when stats=True.  ``out=(src, dst)`` reuses
    buffers (then MH_ECAPACITY raises instead of retrying).  ``stage_events``:
    address of an array of 4 hipEvent_t recorded at the stage boundaries."""
    r = _sample(x, None, seed, replica, seg_work, capacity, stats, out, workspace, stage_events, grid_blocks)
    return (r.src, r.dst, r.stats) if stats else (r.src, r.dst)


def sample_chung_lu(w: torch.Tensor, seed: int = 1, replica: int = 0, seg_work: int = DEFAULT_SEG_WORK,
                    capacity: int | None = None, stats: bool = False, out=None, workspace=None,
                    stage_events=None, grid_blocks: int = 0):
    """One sample of the Chung-Lu model read as probabilities, p = min(w_i w_j, 1)
    (Sec. 2.1), by the Miller-Hagberg chain (Sec. 2.3): (src, dst[, stats])."""
    r = _sample(w, None, seed, replica, seg_work, capacity, stats, out, workspace, stage_events, grid_blocks,
                chung_lu=True)
    return (r.src, r.dst, r.stats) if stats else (r.src, r.dst)


def rank_counts(x: torch.Tensor, model: int = MH_MODEL_UBCM, seed: int = 1, replica: int = 0,
                seg_work: int = DEFAULT_SEG_WORK, out: torch.Tensor | None = None, workspace=None,
                stats: bool = False):
    """One unweighted sample (UBCM, or Chung-Lu with model=MH_MODEL_CHUNG_LU)
    reduced to counts by rank: counts[j] = edges whose endpoint of larger rank
    (in the node order) has rank j.  Returns (counts int32[n], n_edges[, stats])."""
    x = _dev_f64(x, "x")
    n = x.numel()
    L = lib()
    plan = PlanParams(int(seg_work), 0, 0, 0, None)
    wsb = L.mh_workspace_bytes(n, 0, ctypes.byref(plan))
    ws = workspace if workspace is not None and workspace.numel() >= wsb else _workspace(wsb, x.device)
    cnt = out if out is not None else torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
    nedge = ctypes.c_int64(0)
    st = Stats()
    _check(L.mh_sample_rank_counts(_ptr(x), n, int(model), seed, replica, ctypes.byref(plan), _ptr(cnt),
                                   ctypes.byref(nedge), _ptr(ws), ws.numel(), ctypes.byref(st) if stats else None,
                                   _stream(x.device)), "mh_sample_rank_counts")
    return (cnt[:n], int(nedge.value), st.as_dict()) if stats else (cnt[:n], int(nedge.value))


def count_triangles(src: torch.Tensor, dst: torch.Tensor, n: int, workspace=None) -> int:
    """Triangles of the simple undirected graph with these edges (each once)."""
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or not src.is_cuda or src.numel() != dst.numel():
        raise ValueError("src and dst must be CUDA int32 tensors of equal length")
    src, dst = src.contiguous(), dst.contiguous()
    L = lib()
    m = src.numel()
    wsb = L.mh_triangles_workspace_bytes(int(n), m)
    ws = workspace if workspace is not None and workspace.numel() >= wsb else _workspace(wsb, src.device)
    tri = ctypes.c_uint64(0)
    _check(L.mh_count_triangles(_ptr(src), _ptr(dst), m, int(n), ctypes.byref(tri), _ptr(ws), ws.numel(),
                                _stream(src.device)), "mh_count_triangles")
    return int(tri.value)


def sample_weighted(x: torch.Tensor, y: torch.Tensor, seed: int = 1, replica: int = 0,
                    seg_work: int = DEFAULT_SEG_WORK, capacity: int | None = None, stats: bool = False, out=None,
                    workspace=None, stage_events=None, grid_blocks: int = 0):
    """One sample of the weighted model (Sec. 2.5, Alg. 1): (src, dst, w)."""
    r = _sample(x, y, seed, replica, seg_work, capacity, stats, out, workspace, stage_events, grid_blocks)
    return (r.src, r.dst, r.w, r.stats) if stats else (r.src, r.dst, r.w)


def sample_async(x: torch.Tensor, y: torch.Tensor | None, out, workspace: torch.Tensor, seed: int = 1,
                 replica: int = 0, seg_work: int = DEFAULT_SEG_WORK, stage_events=None, grid_blocks: int = 0):
    """Enqueue one sample (unweighted if y is None) on the current stream
    without waiting.  ``out = (src, dst[, w])`` and ``workspace`` (at least
    mh_workspace_bytes) are required and belong to the sample until
    ``sample_result`` has read it back."""
    x = _dev_f64(x, "x")
    if y is not None:
        y = _dev_f64(y, "y")
        if y.shape != x.shape:
            raise ValueError("x and y must have the same shape")
    n = x.numel()
    L = lib()
    plan = PlanParams(int(seg_work), 0, int(grid_blocks), 0, stage_events)
    wsb = L.mh_workspace_bytes(n, 1 if y is not None else 0, ctypes.byref(plan))
    if workspace.numel() < wsb:
        raise ValueError(f"workspace of {workspace.numel()} bytes, {wsb} needed")
    src, dst = out[0], out[1]
    w = out[2] if y is not None else None
    cap = min(src.numel(), dst.numel(), w.numel() if w is not None else src.numel())
    stream = _stream(x.device)
    if y is None:
        status = L.mh_sample_unweighted_async(_ptr(x), n, seed, replica, ctypes.byref(plan), _ptr(src), _ptr(dst),
                                              cap, _ptr(workspace), workspace.numel(), stream)
    else:
        status = L.mh_sample_weighted_async(_ptr(x), _ptr(y), n, seed, replica, ctypes.byref(plan), _ptr(src),
                                            _ptr(dst), _ptr(w), cap, _ptr(workspace), workspace.numel(), stream)
    _check(status, "mh_sample_async")
    return cap


NOALLOC_MAX_NODES = 262144  # MH_NOALLOC_MAX_NODES


def sample_unweighted_noalloc(x: torch.Tensor, out, seed: int = 1, replica: int = 0,
                              seg_work: int = DEFAULT_SEG_WORK, stats: bool = False, grid_blocks: int = 0):
    """mh_sample_unweighted_noalloc: one unweighted sample into the caller's
    ``out = (src, dst)`` with the library's own scratch (no workspace, no
    allocation in the call; n <= NOALLOC_MAX_NODES).  Returns (src, dst) views
    of the edges (and a stats dict when stats=True); MH_ECAPACITY raises."""
    x = _dev_f64(x, "x")
    src, dst = out
    cap = min(src.numel(), dst.numel())
    plan = PlanParams(int(seg_work), 0, int(grid_blocks), 0, None)
    nedge = ctypes.c_int64(0)
    st = Stats()
    _check(lib().mh_sample_unweighted_noalloc(_ptr(x), x.numel(), seed, replica, ctypes.byref(plan), _ptr(src),
                                              _ptr(dst), cap, ctypes.byref(nedge),
                                              ctypes.byref(st) if stats else None, _stream(x.device)),
           "mh_sample_unweighted_noalloc")
    m = int(nedge.value)
    return (src[:m], dst[:m], st.as_dict()) if stats else (src[:m], dst[:m])


def sample_result(workspace: torch.Tensor, capacity: int) -> int:
    """Edge count of the last asynchronous sample of ``workspace`` (waits)."""
    nedge = ctypes.c_int64(0)
    status = lib().mh_sample_result(_ptr(workspace), workspace.numel(), int(capacity), ctypes.byref(nedge),
                                    _stream(workspace.device))
    _check(status, "mh_sample_result")
    return int(nedge.value)


MH_BIP_NO_SELF = 1


def sample_bipartite(x_rows: torch.Tensor, x_cols: torch.Tensor, y_rows: torch.Tensor | None = None,
                     y_cols: torch.Tensor | None = None, exclude_self: bool = False, seed: int = 1, replica: int = 0,
                     seg_work: int = DEFAULT_SEG_WORK, capacity: int | None = None, stats: bool = False, out=None,
                     workspace=None, stage_events=None, grid_blocks: int = 0) -> SampleResult:
    """One sample of a bipartite network (Sec. 2.6): rows = "+" set, columns =
    "-" set; weighted when y_rows and y_cols are given.  exclude_self: directed
    network without self-loops (rows = out-, columns = in-parameters of the
    same nodes).  Returns a SampleResult of (row id, column id[, w])."""
    xr = _dev_f64(x_rows, "x_rows")
    xc = _dev_f64(x_cols, "x_cols")
    if (y_rows is None) != (y_cols is None):
        raise ValueError("give both y_rows and y_cols, or neither")
    weighted = y_rows is not None
    yr = _dev_f64(y_rows, "y_rows") if weighted else None
    yc = _dev_f64(y_cols, "y_cols") if weighted else None
    if weighted and (yr.shape != xr.shape or yc.shape != xc.shape):
        raise ValueError("x and y of a node set must have the same shape")
    nr, nc = xr.numel(), xc.numel()
    dev = xr.device
    L = lib()
    plan = PlanParams(int(seg_work), 0, int(grid_blocks), 0, stage_events)
    wsb = L.mh_bipartite_workspace_bytes(nr, nc, 1 if weighted else 0, ctypes.byref(plan))
    ws = workspace if workspace is not None and workspace.numel() >= wsb else _workspace(wsb, dev)
    cap = int(capacity) if capacity is not None else max(4096, 4 * (nr + nc))
    if out is not None:
        src, dst = out[0], out[1]
        w = out[2] if weighted else None
        cap = min(src.numel(), dst.numel(), w.numel() if w is not None else src.numel())
    else:
        src = dst = w = None
    flags = MH_BIP_NO_SELF if exclude_self else 0
    nedge = ctypes.c_int64(0)
    st = Stats()
    for _attempt in range(2):
        if src is None or src.numel() < cap:
            src = torch.empty(cap, dtype=torch.int32, device=dev)
            dst = torch.empty(cap, dtype=torch.int32, device=dev)
            w = torch.empty(cap, dtype=torch.int32, device=dev) if weighted else None
        status = L.mh_sample_bipartite(_ptr(xr), _ptr(yr), nr, _ptr(xc), _ptr(yc), nc, flags, seed, replica,
                                       ctypes.byref(plan), _ptr(src), _ptr(dst), _ptr(w), cap, ctypes.byref(nedge),
                                       _ptr(ws), ws.numel(), ctypes.byref(st) if stats else None, _stream(dev))
        if status == MH_ECAPACITY and out is None:
            cap = int(nedge.value)
            src = None
            continue
        _check(status, "mh_sample_bipartite")
        break
    m = int(nedge.value)
    return SampleResult(src[:m], dst[:m], None if w is None else w[:m], st.as_dict() if stats else None)


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
    plan = PlanParams(DEFAULT_SEG_WORK, 0, 0, 0, None)
    ws = _workspace(L.mh_workspace_bytes(n, 1 if y is not None else 0, ctypes.byref(plan)), dev)
    _check(L.mh_order(_ptr(x), _ptr(y), n, _ptr(perm), _ptr(zs), _ptr(ys), _ptr(status), _ptr(ws), ws.numel(),
                      _stream(dev)), "mh_order")
    return perm, zs, ys, status


def sort_edges(src: torch.Tensor, dst: torch.Tensor, w: torch.Tensor | None = None, workspace=None):
    """Sorts an edge list in place into canonical order, by (src, dst) (node
    ids; the method's edge list is a set, so this order makes samples
    comparable element by element).  Returns (src, dst, w)."""
    if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.shape != dst.shape or not src.is_cuda:
        raise ValueError("src and dst must be int32 device tensors of one shape")
    if w is not None and (w.dtype != torch.int32 or w.shape != src.shape):
        raise ValueError("w must be an int32 tensor of the edges' shape")
    if not (src.is_contiguous() and dst.is_contiguous() and (w is None or w.is_contiguous())):
        raise ValueError("edge arrays must be contiguous")
    L = lib()
    m = src.numel()
    need = L.mh_sort_edges_workspace_bytes(m)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, src.device)
    _check(L.mh_sort_edges(_ptr(src), _ptr(dst), _ptr(w), m, _ptr(ws), ws.numel(), _stream(src.device)),
           "mh_sort_edges")
    return src, dst, w


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


# ---------------------------------------------------------------------------- batched ensembles
MH_BATCH_EDGES, MH_BATCH_DEGREES, MH_BATCH_DEGREES_STAGED = 0, 1, 2
BATCH_EDGE_SLACK = 4096 * 4096  # MH_BATCH_EDGE_SLACK: room beyond the edges for the waves' output chunks


class Network(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("seg_work", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("seg_work", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("ms", ctypes.c_float)]


def _batch_sigs(L):
    if getattr(L, "_batch_ready", False):
        return
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "mh_batch_workspace_bytes": ([vp, i32, i32], sz),
        "mh_batch_prepare": ([vp, i32, i32, vp, sz, vp], ctypes.c_int),
        "mh_batch_sample_async": ([vp, i32, i32, vp, sz, vp, vp, i32, u64, i32, vp, vp, vp, vp, i64, vp, vp, i32, vp],
                                  ctypes.c_int),
        "mh_batch_result": ([vp, i32, i32, vp, sz, P(i64), i64, vp], ctypes.c_int),
        "mh_batch_capture": ([vp, i32, i32, vp, sz, vp, vp, i32, u64, i32, vp, vp, vp, vp, i64, vp, vp, i32, vp,
                              P(vp)], ctypes.c_int),
        "mh_batch_autotune": ([vp, i32, i32, vp, sz, vp, vp, i32, vp, vp, vp, i32, vp, i32, P(Tuning), vp],
                              ctypes.c_int),
        "mh_graph_launch": ([vp, vp], ctypes.c_int),
        "mh_graph_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    L._batch_ready = True


class Batch:
    """Prepared ensemble of networks (A1-A3 done once) sampled by one persistent launch.

    xs: list of float64 CUDA tensors (one per network); ys: same-length list for
    the weighted model, or None.  Sample (i, r) equals sample_unweighted(xs[i],
    seed, r, seg_work) edge for edge."""

    def __init__(self, xs, ys=None, seg_work: int | list = DEFAULT_SEG_WORK, max_samples: int = 4096):
        L = lib()
        _batch_sigs(L)
        self.L = L
        self.xs = [_dev_f64(x, "x") for x in xs]
        self.ys = None if ys is None else [_dev_f64(y, "y") for y in ys]
        self.device = self.xs[0].device
        k = len(self.xs)
        sw = [int(seg_work)] * k if not isinstance(seg_work, (list, tuple)) else [int(v) for v in seg_work]
        self.nets = (Network * k)()
        for i, x in enumerate(self.xs):
            self.nets[i].n = x.numel()
            self.nets[i].x = x.data_ptr()
            self.nets[i].y = None if self.ys is None else self.ys[i].data_ptr()
            self.nets[i].seg_work = sw[i]
        self.k = k
        self.max_samples = int(max_samples)
        self.sizes = [x.numel() for x in self.xs]
        self.ws = _workspace(self._ws_bytes(), self.device)
        _check(L.mh_batch_prepare(self.nets, k, self.max_samples, _ptr(self.ws), self.ws.numel(),
                                  _stream(self.device)), "mh_batch_prepare")

    def _ws_bytes(self):
        return self.L.mh_batch_workspace_bytes(self.nets, self.k, self.max_samples)

    def _refs(self, sample_net, sample_rep):
        net = torch.as_tensor(sample_net, dtype=torch.int32, device=self.device).contiguous()
        rep = torch.as_tensor(sample_rep, dtype=torch.int64, device=self.device).to(torch.int32).contiguous()
        if net.numel() != rep.numel() or net.numel() > self.max_samples:
            raise ValueError("sample lists must have equal length <= max_samples")
        return net, rep

    def degree_offsets(self, sample_net):
        # an index outside the batch sizes as 0 here; the library rejects it
        sizes = torch.as_tensor([self.sizes[int(i)] if 0 <= int(i) < self.k else 0
                                 for i in torch.as_tensor(sample_net).tolist()], dtype=torch.int64)
        off = torch.zeros(len(sizes) + 1, dtype=torch.int64)
        off[1:] = torch.cumsum(sizes, 0)
        return off

    def sample_edges_async(self, net, rep, seed, src, dst, w, sid, capacity, grid_blocks=0):
        _check(self.L.mh_batch_sample_async(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(),
                                            _ptr(net), _ptr(rep), net.numel(), seed, MH_BATCH_EDGES, _ptr(src),
                                            _ptr(dst), _ptr(w), _ptr(sid), capacity, None, None, grid_blocks,
                                            _stream(self.device)), "mh_batch_sample_async")

    def result(self, capacity=-1) -> int:
        m = ctypes.c_int64(0)
        st = self.L.mh_batch_result(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(),
                                    ctypes.byref(m), capacity, _stream(self.device))
        if st not in (MH_OK, MH_ECAPACITY):
            _check(st, "mh_batch_result")
        return int(m.value) if st == MH_OK else -int(m.value)

    def sample_edges(self, sample_net, sample_rep, seed: int = 1, capacity: int | None = None, grid_blocks=0):
        """(src, dst, w|None, sid) of every listed sample, order unspecified.
        capacity: output slots; the call needs the edges plus a chunk of
        MH_BATCH_OUT_CHUNK slots per wave of the launch (BATCH_EDGE_SLACK always
        suffices), and retries once with the capacity the library reports."""
        net, rep = self._refs(sample_net, sample_rep)
        cap = int(capacity) if capacity is not None else max(
            4096, 4 * sum(self.sizes[i] for i in net.tolist() if 0 <= i < self.k)) + BATCH_EDGE_SLACK
        for _ in range(2):
            src = torch.empty(cap, dtype=torch.int32, device=self.device)
            dst = torch.empty(cap, dtype=torch.int32, device=self.device)
            w = torch.empty(cap, dtype=torch.int32, device=self.device) if self.ys is not None else None
            sid = torch.empty(cap, dtype=torch.int32, device=self.device)
            self.sample_edges_async(net, rep, seed, src, dst, w, sid, cap, grid_blocks)
            m = self.result(cap)
            if m >= 0:
                return src[:m], dst[:m], (None if w is None else w[:m]), sid[:m]
            cap = -m
        raise MHError(MH_ECAPACITY, "mh_batch_sample_async")

    def sample_degrees(self, sample_net, sample_rep, seed: int = 1, out=None, grid_blocks=0, slots=None):
        """Concatenated per-sample degree sequences and their offsets (int64, len n_samples + 1).
        slots: an int32 CUDA tensor (scratch) to count the columns through
        (MH_BATCH_DEGREES_STAGED), else every edge adds by a device atomic."""
        net, rep = self._refs(sample_net, sample_rep)
        off = self.degree_offsets(net.cpu())
        deg = out if out is not None else torch.empty(int(off[-1]), dtype=torch.int32, device=self.device)
        offd = off.to(self.device)
        mode, cap = self._degree_mode(slots)
        _check(self.L.mh_batch_sample_async(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(),
                                            _ptr(net), _ptr(rep), net.numel(), seed, mode, _ptr(slots), None,
                                            None, None, cap, _ptr(deg), _ptr(offd), grid_blocks, _stream(self.device)),
               "mh_batch_sample_async")
        self.result(-1)
        return deg, off

    @staticmethod
    def _degree_mode(slots):
        if slots is None:
            return MH_BATCH_DEGREES, 0
        if slots.dtype != torch.int32 or not slots.is_cuda or not slots.is_contiguous():
            raise ValueError("slots must be a contiguous int32 CUDA tensor")
        return MH_BATCH_DEGREES_STAGED, slots.numel()

    def capture_degrees(self, net, rep, seed, deg, offd, grid_blocks=0, slots=None):
        """hipGraph of one degree-sink batch launch; returns a BatchGraph (replay with .launch())."""
        exe = ctypes.c_void_p()
        mode, cap = self._degree_mode(slots)
        _check(self.L.mh_batch_capture(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(), _ptr(net),
                                       _ptr(rep), net.numel(), seed, mode, _ptr(slots), None, None, None, cap,
                                       _ptr(deg), _ptr(offd), grid_blocks, _stream(self.device), ctypes.byref(exe)),
               "mh_batch_capture")
        return BatchGraph(self.L, exe, self.device, keep=(net, rep, deg, offd, slots, self.ws))

    def capture_edges(self, net, rep, seed, src, dst, w, sid, capacity, grid_blocks=0):
        exe = ctypes.c_void_p()
        _check(self.L.mh_batch_capture(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(), _ptr(net),
                                       _ptr(rep), net.numel(), seed, MH_BATCH_EDGES, _ptr(src), _ptr(dst), _ptr(w),
                                       _ptr(sid), capacity, None, None, grid_blocks, _stream(self.device),
                                       ctypes.byref(exe)), "mh_batch_capture")
        return BatchGraph(self.L, exe, self.device, keep=(net, rep, src, dst, w, sid, self.ws))

    def autotune(self, probe_net, probe_rep, seg_candidates=(4, 8, 16, 32), grid_candidates=(0,)):
        """Pick seg_work and grid size on a probe batch (degree sink); re-prepares with the winner."""
        net, rep = self._refs(probe_net, probe_rep)
        off = self.degree_offsets(net.cpu())
        deg = torch.empty(int(off[-1]), dtype=torch.int32, device=self.device)
        offd = off.to(self.device)
        segs = (ctypes.c_int32 * len(seg_candidates))(*seg_candidates)
        grids = (ctypes.c_int32 * len(grid_candidates))(*grid_candidates)
        best = Tuning()
        # the workspace must fit every candidate's layout: size it for the largest
        need = 0
        for sw in seg_candidates:
            for i in range(self.k):
                self.nets[i].seg_work = int(sw)
            need = max(need, self._ws_bytes())
        if self.ws.numel() < need:
            self.ws = _workspace(need, self.device)
        _check(self.L.mh_batch_autotune(self.nets, self.k, self.max_samples, _ptr(self.ws), self.ws.numel(), _ptr(net),
                                        _ptr(rep), net.numel(), _ptr(deg), _ptr(offd), segs, len(seg_candidates),
                                        grids, len(grid_candidates), ctypes.byref(best), _stream(self.device)),
               "mh_batch_autotune")
        return {"seg_work": best.seg_work, "grid_blocks": best.grid_blocks, "ms": best.ms}


class BatchGraph:
    """An executable hipGraph of one batch launch.  It holds the tensors whose
    device addresses the graph captured, so they outlive every replay."""

    def __init__(self, L, exe, device, keep=()):
        self.L, self.exe, self.device = L, exe, device
        self._keep = keep

    def launch(self):
        _check(self.L.mh_graph_launch(self.exe, _stream(self.device)), "mh_graph_launch")

    def __del__(self):
        try:
            if self.exe:
                self.L.mh_graph_destroy(self.exe)
        except Exception:
            pass
