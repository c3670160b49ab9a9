"""CPU oracle for the UBCM / UECM Miller-Hagberg samplers.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (``paper_2509_13230_amd``) and never imports it.

The arithmetic lives in ``mh_oracle.c`` (plain C, binary64, no contraction);
this module compiles it on first use and wraps it with ctypes.  The exact
path-tree enumeration used to pin the algorithm lives in ``enumerate.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mh_oracle.c")
_HDR = os.path.join(_HERE, "mh_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add, every operation rounds once.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = False) -> str:
    """Compile liboracle.so next to its source (gcc)."""
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(p) > os.path.getmtime(_LIB) for p in (_SRC, _HDR)
    )
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path = None  # another build of mh_oracle.c to load instead (see use_library)


def use_library(path: str) -> None:
    """Load the oracle's functions from another build of its source from now
    on (the planted-mistake test builds altered copies of mh_oracle.c)."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = _lib_path if _lib_path is not None else build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i32, i64, u32, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        vp = ctypes.c_void_p
        L.mho_philox4x32_10.argtypes = [vp, vp, vp]
        L.mho_philox4x32_10.restype = None
        L.mho_u53.argtypes = [u32, u32]
        L.mho_u53.restype = d
        L.mho_skip_real.argtypes = [d, d, d]
        L.mho_skip_real.restype = d
        L.mho_skip_reals.argtypes = [vp, i64, d, d, vp]
        L.mho_skip_reals.restype = None
        L.mho_order.argtypes = [vp, i64, vp]
        L.mho_bound.argtypes = [vp, i64, vp]
        L.mho_plan_counts.argtypes = [vp, vp, i64, i32, vp]
        L.mho_plan_row.argtypes = [vp, vp, i64, i32, i64, vp, vp, i64]
        L.mho_plan_row.restype = i64
        L.mho_sample_mh.argtypes = [vp, vp, i64, u64, u32, i32, vp, vp, vp, i64, vp, vp, i64, P(i64)]
        L.mho_sample_mh.restype = i64
        L.mho_sample_bipartite.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, u64, u32, i32, vp, vp, vp, i64,
                                           vp, vp, i64, P(i64)]
        L.mho_sample_bipartite.restype = i64
        L.mho_sample_bipartite_bf.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, u64, u32, vp, vp, vp, i64]
        L.mho_sample_bipartite_bf.restype = i64
        L.mho_plan_row_bipartite.argtypes = [vp, i64, d, d, i32, vp, vp, i64]
        L.mho_plan_row_bipartite.restype = i64
        L.mho_sample_chung_lu.argtypes = [vp, i64, u64, u32, i32, vp, vp, i64, vp, vp, i64, P(i64)]
        L.mho_sample_chung_lu.restype = i64
        L.mho_count_triangles.argtypes = [vp, vp, i64, i64]
        L.mho_count_triangles.restype = i64
        L.mho_sample_bf.argtypes = [vp, vp, i64, u64, u32, i64, i64, vp, vp, vp, i64, P(i64)]
        L.mho_sample_bf.restype = i64
        L.mho_expected_degree.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
        L.mho_expected_degree_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
        _lib = L
    return _lib


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("steps", "proposals", "accepts", "segments", "saturated_w", "near_ties")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().mho_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def u53(a: int, b: int) -> float:
    return lib().mho_u53(a, b)


def skip_reals(u1, tq: float, c: float = 1.0) -> np.ndarray:
    """The sampler's skip d = -log(u1) / log1p(tq / c) for each uniform u1
    (the candidate is floor(d) columns past the chain's position)."""
    u = _f64(u1)
    d = np.zeros(len(u))
    lib().mho_skip_reals(_p(u), len(u), float(tq), float(c), _p(d))
    return d


def order(z) -> np.ndarray:
    z = _f64(z)
    perm = np.zeros(len(z), dtype=np.int32)
    lib().mho_order(_p(z), len(z), _p(perm))
    return perm


def bound(ys) -> np.ndarray:
    ys = _f64(ys)
    c = np.zeros(len(ys), dtype=np.float64)
    lib().mho_bound(_p(ys), len(ys), _p(c))
    return c


def sorted_params(x, y=None):
    """(perm, zs, ys, c): the node order and the sorted arrays the sweep reads."""
    x = _f64(x)
    z = x if y is None else x * _f64(y)
    perm = order(z)
    zs = z[perm]
    ys = None if y is None else _f64(y)[perm]
    c = None if y is None else bound(ys)
    return perm, zs, ys, c


def plan_counts(zs, c, seg_work: int) -> np.ndarray:
    zs = _f64(zs)
    c = _f64(c)
    out = np.zeros(len(zs), dtype=np.int32)
    lib().mho_plan_counts(_p(zs), _p(c), len(zs), seg_work, _p(out))
    return out


def plan_row(zs, c, seg_work: int, r: int):
    zs = _f64(zs)
    c = _f64(c)
    cnt = lib().mho_plan_row(_p(zs), _p(c), len(zs), seg_work, r, None, None, 0)
    a = np.zeros(max(cnt, 1), dtype=np.int64)
    b = np.zeros(max(cnt, 1), dtype=np.int64)
    lib().mho_plan_row(_p(zs), _p(c), len(zs), seg_work, r, _p(a), _p(b), cnt)
    return a[:cnt], b[:cnt]


@dataclass
class Sample:
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray | None
    stats: dict
    tie_rows: np.ndarray

    @property
    def n_edges(self) -> int:
        return len(self.src)


def sample_mh(x, y=None, seed: int = 1, replica: int = 0, seg_work: int = 0,
              capacity: int | None = None) -> Sample:
    """Sequential sampler (UBCM if y is None, else UECM)."""
    x = _f64(x)
    y = _f64(y)
    n = len(x)
    st = Stats()
    ntr = ctypes.c_int64(0)
    cap = capacity if capacity is not None else max(1024, 8 * n)
    tcap = 1024
    while True:
        src = np.zeros(cap, dtype=np.int32)
        dst = np.zeros(cap, dtype=np.int32)
        w = np.zeros(cap, dtype=np.int32) if y is not None else None
        ties = np.zeros(tcap, dtype=np.int32)
        m = lib().mho_sample_mh(_p(x), _p(y), n, seed, replica, seg_work, _p(src), _p(dst), _p(w), cap,
                                ctypes.byref(st), _p(ties), len(ties), ctypes.byref(ntr))
        if m < 0:
            raise ValueError("oracle: invalid parameters (code %d)" % m)
        if m <= cap and ntr.value <= tcap:
            break
        cap, tcap = max(cap, int(m)), max(tcap, int(ntr.value))
    return Sample(src[:m], dst[:m], None if w is None else w[:m], st.as_dict(), ties[: ntr.value].copy())


def sample_chung_lu(w, seed: int = 1, replica: int = 0, seg_work: int = 0, capacity: int | None = None) -> Sample:
    """Miller-Hagberg sampler of the Chung-Lu model, p_ij = min(w_i w_j, 1)
    (Sec. 2.3; the biased comparison model of Sec. 2.1)."""
    w = _f64(w)
    n = len(w)
    st = Stats()
    ntr = ctypes.c_int64(0)
    cap = capacity if capacity is not None else max(1024, 8 * n)
    tcap = 1024
    while True:
        src = np.zeros(cap, dtype=np.int32)
        dst = np.zeros(cap, dtype=np.int32)
        ties = np.zeros(tcap, dtype=np.int32)
        m = lib().mho_sample_chung_lu(_p(w), n, seed, replica, seg_work, _p(src), _p(dst), cap, ctypes.byref(st),
                                      _p(ties), len(ties), ctypes.byref(ntr))
        if m < 0:
            raise ValueError("oracle: invalid parameters (code %d)" % m)
        if m <= cap and ntr.value <= tcap:
            break
        cap, tcap = max(cap, int(m)), max(tcap, int(ntr.value))
    return Sample(src[:m], dst[:m], None, st.as_dict(), ties[: ntr.value].copy())


def count_triangles(src, dst, n: int) -> int:
    """Triangles of the simple undirected graph with these edges (each once)."""
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    t = lib().mho_count_triangles(_p(s), _p(d), len(s), int(n))
    if t < 0:
        raise ValueError("oracle: invalid edge list")
    return int(t)


def rank_counts(src, dst, perm) -> np.ndarray:
    """counts[j] = number of edges whose endpoint of larger rank (later in the
    node order perm) has rank j: the edges among the first K ranks number
    counts[:K].sum(), the numerator of the rich-club density of the K nodes of
    largest parameter (Sec. 2.1, Fig. 1A)."""
    perm = np.asarray(perm)
    rank = np.empty(len(perm), dtype=np.int64)
    rank[perm] = np.arange(len(perm))
    hi = np.maximum(rank[np.asarray(src, np.int64)], rank[np.asarray(dst, np.int64)])
    return np.bincount(hi, minlength=len(perm)).astype(np.int64)


def sample_bf(x, y=None, seed: int = 1, replica: int = 0, row_begin: int = 0, row_end: int | None = None,
              capacity: int | None = None):
    """Brute-force Bernoulli sampler over pairs i<j, i in [row_begin, row_end)."""
    x = _f64(x)
    y = _f64(y)
    n = len(x)
    re = n if row_end is None else row_end
    cap = capacity if capacity is not None else max(1024, 8 * n)
    ties = ctypes.c_int64(0)
    while True:
        src = np.zeros(cap, dtype=np.int32)
        dst = np.zeros(cap, dtype=np.int32)
        w = np.zeros(cap, dtype=np.int32) if y is not None else None
        m = lib().mho_sample_bf(_p(x), _p(y), n, seed, replica, row_begin, re, _p(src), _p(dst), _p(w), cap,
                                ctypes.byref(ties))
        if m < 0:
            raise ValueError("oracle: invalid parameters (code %d)" % m)
        if m <= cap:
            break
        cap = int(m)
    return src[:m], dst[:m], (None if w is None else w[:m]), ties.value


def expected_degree(x, y=None, mult=None, rows=None):
    x = _f64(x)
    y = _f64(y)
    mult = _f64(mult)
    n = len(x)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if r is None else len(r)
    k = np.zeros(cnt)
    s = np.zeros(cnt) if y is not None else None
    lib().mho_expected_degree(_p(x), _p(y), _p(mult), n, _p(r), cnt, _p(k), _p(s))
    return k, s


def expected_degree_grad(x, y=None, mult=None, gk=None, gs=None):
    x = _f64(x)
    y = _f64(y)
    mult = _f64(mult)
    n = len(x)
    gk = _f64(gk if gk is not None else np.zeros(n))
    gs = _f64(gs) if (y is not None) else None
    if y is not None and gs is None:
        gs = np.zeros(n)
    gx = np.zeros(n)
    gy = np.zeros(n) if y is not None else None
    lib().mho_expected_degree_grad(_p(x), _p(y), _p(mult), n, _p(gk), _p(gs), _p(gx), _p(gy))
    return gx, gy


def sample_bipartite(xr, xc, yr=None, yc=None, exclude_self=False, seed: int = 1, replica: int = 0,
                     seg_work: int = 0, capacity: int | None = None) -> Sample:
    """Bipartite (rows = "+" set, columns = "-" set) or, with exclude_self,
    directed sampler (rows = out-parameters, columns = in-parameters)."""
    xr, xc, yr, yc = _f64(xr), _f64(xc), _f64(yr), _f64(yc)
    st = Stats()
    ntr = ctypes.c_int64(0)
    cap = capacity if capacity is not None else max(1024, 8 * (len(xr) + len(xc)))
    tcap = 1024
    while True:
        src = np.zeros(cap, dtype=np.int32)
        dst = np.zeros(cap, dtype=np.int32)
        w = np.zeros(cap, dtype=np.int32) if yr is not None else None
        ties = np.zeros(tcap, dtype=np.int32)
        m = lib().mho_sample_bipartite(_p(xr), _p(yr), len(xr), _p(xc), _p(yc), len(xc), int(exclude_self), seed,
                                       replica, seg_work, _p(src), _p(dst), _p(w), cap, ctypes.byref(st), _p(ties),
                                       len(ties), ctypes.byref(ntr))
        if m < 0:
            raise ValueError("oracle: invalid parameters (code %d)" % m)
        if m <= cap and ntr.value <= tcap:
            break
        cap, tcap = max(cap, int(m)), max(tcap, int(ntr.value))
    return Sample(src[:m], dst[:m], None if w is None else w[:m], st.as_dict(), ties[: ntr.value].copy())


def sample_bipartite_bf(xr, xc, yr=None, yc=None, exclude_self=False, seed: int = 1, replica: int = 0,
                        capacity: int | None = None):
    xr, xc, yr, yc = _f64(xr), _f64(xc), _f64(yr), _f64(yc)
    cap = capacity if capacity is not None else max(1024, len(xr) * len(xc))
    src = np.zeros(cap, dtype=np.int32)
    dst = np.zeros(cap, dtype=np.int32)
    w = np.zeros(cap, dtype=np.int32) if yr is not None else None
    m = lib().mho_sample_bipartite_bf(_p(xr), _p(yr), len(xr), _p(xc), _p(yc), len(xc), int(exclude_self), seed,
                                      replica, _p(src), _p(dst), _p(w), cap)
    if m < 0:
        raise ValueError("oracle: invalid parameters (code %d)" % m)
    return src[:m], dst[:m], (None if w is None else w[:m])


def plan_row_bipartite(zcs, s: float, c: float, seg_work: int):
    """Column segments [a_k, b_k) of one bipartite row (value s, bound c)."""
    zcs = _f64(zcs)
    cnt = lib().mho_plan_row_bipartite(_p(zcs), len(zcs), s, c, seg_work, None, None, 0)
    a = np.zeros(max(cnt, 1), dtype=np.int64)
    b = np.zeros(max(cnt, 1), dtype=np.int64)
    lib().mho_plan_row_bipartite(_p(zcs), len(zcs), s, c, seg_work, _p(a), _p(b), cnt)
    return a[:cnt], b[:cnt]
