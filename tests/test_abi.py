"""Host-side checks of the C-ABI library: it loads, exports every symbol that
include/mh.h declares, and its argument checks fail before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mh.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mh_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2509_13230_amd as mh

    if not os.path.exists(mh.library_path()):
        mh_build = pytest.importorskip("paper_2509_13230_amd.build")
        mh_build.build(verbose=False)
    return mh.lib()


def test_header_declares_entry_points():
    names = _declared()
    for must in ("mh_sample_unweighted", "mh_sample_weighted", "mh_sample_bruteforce", "mh_expected_degree_fwd",
                 "mh_expected_degree_bwd", "mh_order", "mh_bound", "mh_plan_counts", "mh_workspace_bytes",
                 "mh_sample_bipartite", "mh_bipartite_workspace_bytes", "mh_sort_edges",
                 "mh_sort_edges_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_workspace_sizes_grow_with_n(L):
    import paper_2509_13230_amd as mh

    p = mh.PlanParams(32, 0, 0, 0, None)
    a = L.mh_workspace_bytes(1000, 0, ctypes.byref(p))
    b = L.mh_workspace_bytes(1_000_000, 0, ctypes.byref(p))
    c = L.mh_workspace_bytes(1_000_000, 1, ctypes.byref(p))
    assert 0 < a < b < c
    # roughly linear: a few hundred bytes per node (most of it room for the
    # records of up to 8 heavy items per row)
    assert b < 400 * 1_000_000
    assert L.mh_bruteforce_workspace_bytes(50_000) > 0


def test_null_plan_means_documented_default(L):
    import paper_2509_13230_amd as mh

    p = mh.PlanParams(mh.DEFAULT_SEG_WORK, 0, 0, 0, None)
    for n in (1000, 1_000_000):
        assert L.mh_workspace_bytes(n, 1, None) == L.mh_workspace_bytes(n, 1, ctypes.byref(p))
        assert L.mh_bipartite_workspace_bytes(n, 777, 1, None) == L.mh_bipartite_workspace_bytes(
            n, 777, 1, ctypes.byref(p))
    assert mh.DEFAULT_SEG_WORK == 8  # the value include/mh.h documents for a NULL plan
    assert "NULL = {seg_work = 8" in open(HEADER).read()


def test_argument_errors_return_before_device_work(L):
    n = ctypes.c_int64(0)
    # missing n_edges_host
    assert L.mh_sample_unweighted(None, 10, 1, 0, None, None, None, 0, None, None, 0, None, None) == -1
    # negative n
    assert L.mh_sample_unweighted(None, -1, 1, 0, None, None, None, 0, ctypes.byref(n), None, 0, None, None) == -1
    # n = 0 is an empty sample
    assert L.mh_sample_unweighted(None, 0, 1, 0, None, None, None, 0, ctypes.byref(n), None, 0, None, None) == 0
    assert n.value == 0
    # capacity > 0 needs output pointers
    assert L.mh_sample_unweighted(ctypes.c_void_p(16), 10, 1, 0, None, None, None, 5, ctypes.byref(n), None, 0,
                                  None, None) == -1
    # workspace too small
    assert L.mh_sample_unweighted(ctypes.c_void_p(16), 10, 1, 0, None, ctypes.c_void_p(16), ctypes.c_void_p(16), 5,
                                  ctypes.byref(n), None, 0, None, None) == -4
    # negative plan parameter
    import paper_2509_13230_amd as mh

    bad = mh.PlanParams(-3, 0, 0, 0, None)
    assert L.mh_sample_unweighted(ctypes.c_void_p(16), 10, 1, 0, ctypes.byref(bad), ctypes.c_void_p(16),
                                  ctypes.c_void_p(16), 5, ctypes.byref(n), ctypes.c_void_p(256), 1 << 20, None,
                                  None) == -1
    assert L.mh_status_string(-2) == b"output capacity too small"


def test_bipartite_argument_errors(L):
    import paper_2509_13230_amd as mh

    n = ctypes.c_int64(7)
    P = ctypes.c_void_p(16)
    ws = ctypes.c_void_p(256)

    def call(xr, yr, nr, xc, yc, nc, flags=0, plan=None, cap=0, src=None, dst=None, w=None, nptr=ctypes.byref(n),
             workspace=None, wsb=0):
        return L.mh_sample_bipartite(xr, yr, nr, xc, yc, nc, flags, 1, 0, plan, src, dst, w, cap, nptr, workspace,
                                     wsb, None, None)

    assert call(P, None, 10, P, None, 10, nptr=None) == -1           # no n_edges_host
    assert call(P, None, -1, P, None, 10) == -1                      # negative size
    assert call(P, P, 10, P, None, 10) == -1                         # one y missing
    assert call(P, None, 10, P, None, 10, flags=2) == -1             # unknown flag
    assert call(None, None, 10, P, None, 10) == -1                   # no row parameters
    assert call(P, None, 10, P, None, 10, cap=5) == -1               # capacity without outputs
    bad = mh.PlanParams(-1, 0, 0, 0, None)
    assert call(P, None, 10, P, None, 10, plan=ctypes.byref(bad)) == -1
    assert call(P, None, 10, P, None, 10, workspace=ws, wsb=1024) == -4  # workspace too small
    assert call(None, None, 0, P, None, 10) == 0 and n.value == 0    # an empty set: empty sample
    n.value = 7
    assert call(P, None, 10, None, None, 0) == 0 and n.value == 0
    p = mh.PlanParams(16, 0, 0, 0, None)
    a = L.mh_bipartite_workspace_bytes(1000, 2000, 0, ctypes.byref(p))
    b = L.mh_bipartite_workspace_bytes(1_000_000, 2000, 0, ctypes.byref(p))
    c = L.mh_bipartite_workspace_bytes(1_000_000, 2000, 1, ctypes.byref(p))
    assert 0 < a < b < c < 400 * 1_002_000


def test_binding_fails_loudly_without_device():
    import torch

    import paper_2509_13230_amd as mh

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(TypeError):
        mh.sample_unweighted(torch.zeros(10, dtype=torch.float64))


def test_sort_edges_argument_errors(L):
    P = ctypes.c_void_p(16)
    assert L.mh_sort_edges(None, None, None, -1, None, 0, None) == -1           # negative count
    assert L.mh_sort_edges(None, None, None, 1 << 31, None, 0, None) == -1      # beyond INT32_MAX edges
    assert L.mh_sort_edges(None, None, None, 0, None, 0, None) == 0             # nothing to sort
    assert L.mh_sort_edges(None, None, None, 1, None, 0, None) == 0
    assert L.mh_sort_edges(None, P, None, 10, P, 1 << 20, None) == -1           # no src
    assert L.mh_sort_edges(P, P, None, 10, P, 16, None) == -4                   # workspace too small
    a = L.mh_sort_edges_workspace_bytes(1000)
    b = L.mh_sort_edges_workspace_bytes(1_000_000)
    assert 0 < a < b < 40 * 1_000_000


def test_probe_library_exports_and_checks_arguments(L):
    """The benchmark's atomic-rate probe lives in a library of its own; its
    argument checks (power-of-two table, positive grid) return before any
    device work."""
    import paper_2509_13230_amd as mh

    path = os.path.join(os.path.dirname(mh.library_path()), "libmh_probe.so")
    P = ctypes.CDLL(path)
    f = P.mhp_atomic_adds
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    assert not hasattr(L, "mhp_atomic_adds")
    fake = ctypes.c_void_p(0x1000)
    assert f(None, 1024, 1, 1, None) == -1
    assert f(fake, 1000, 1, 1, None) == -1
    assert f(fake, 0, 1, 1, None) == -1
    assert f(fake, 1 << 31, 1, 1, None) == -1
    assert f(fake, 1024, 0, 1, None) == -1
    assert f(fake, 1024, 1, -1, None) == -1


def test_binding_constants_match_header():
    # the binding restates a few of the header's values; they must agree
    import re

    import paper_2509_13230_amd as mh

    hdr = open(os.path.join(ROOT, "include", "mh.h")).read()

    def define(name):
        m = re.search(r"#define\s+" + name + r"\s+\(?([0-9]+)(?:ll)?(?:\s*\*\s*([0-9]+)(?:ll)?)?\)?", hdr)
        assert m, name
        return int(m.group(1)) * (int(m.group(2)) if m.group(2) else 1)

    assert define("MH_BATCH_EDGES") == mh.MH_BATCH_EDGES
    assert define("MH_BATCH_DEGREES") == mh.MH_BATCH_DEGREES
    assert define("MH_BATCH_DEGREES_STAGED") == mh.MH_BATCH_DEGREES_STAGED
    assert define("MH_BATCH_EDGE_SLACK") == mh.BATCH_EDGE_SLACK
    # a chunk per wave, at most 4096 waves a launch
    assert define("MH_BATCH_EDGE_SLACK") == define("MH_BATCH_OUT_CHUNK") * 4096
    assert define("MH_NOALLOC_MAX_NODES") == mh.NOALLOC_MAX_NODES
