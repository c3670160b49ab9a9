"""The allocation-free sampler (mh_sample_unweighted_noalloc) against the
sampler with a caller workspace (mh_sample_unweighted), through the C-ABI:
two calls in a row, the second on a smaller network, each identical to the
workspace sampler's sample edge for edge and counter for counter; sizes
beyond the scratch are rejected before any device work."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mh():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2509_13230_amd as m

    m.lib()
    return m


def _keys(src, dst, n):
    return np.sort(src.cpu().numpy().astype(np.int64) * n + dst.cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("seg_work", [8, 0])
def test_noalloc_matches_workspace_sampler(mh, seg_work):
    rng = np.random.default_rng(31)
    big = workloads.chung_lu_scale(workloads.powerlaw_degrees(rng, mh.NOALLOC_MAX_NODES, 2.1, 1, 3000))
    small = workloads.lognormal_x(rng, 5000, -4.0, 1.5)
    cap = 4_000_000
    out = (torch.empty(cap, dtype=torch.int32, device="cuda"), torch.empty(cap, dtype=torch.int32, device="cuda"))
    for x, replica in ((big, 3), (small, 4)):
        xd = torch.as_tensor(x).cuda()
        s1, d1, st1 = mh.sample_unweighted_noalloc(xd, out, seed=7, replica=replica, seg_work=seg_work, stats=True)
        s2, d2, st2 = mh.sample_unweighted(xd, seed=7, replica=replica, seg_work=seg_work, stats=True)
        assert len(s1) > 0
        assert np.array_equal(_keys(s1, d1, len(x)), _keys(s2, d2, len(x)))
        assert st1 == st2


def test_noalloc_rejects_sizes_beyond_scratch(mh):
    L = mh.lib()
    n = mh.NOALLOC_MAX_NODES + 1
    x = torch.full((n,), 0.01, dtype=torch.float64, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    nedge = ctypes.c_int64(-1)
    plan = mh.PlanParams(8, 0, 0, 0, None)
    st = L.mh_sample_unweighted_noalloc(x.data_ptr(), n, 1, 0, ctypes.byref(plan), out.data_ptr(), out.data_ptr(),
                                        16, ctypes.byref(nedge), None, None)
    assert st == mh.MH_EINVAL and nedge.value == 0


def test_noalloc_capacity_is_reported(mh):
    x = torch.as_tensor(workloads.cfg1_small(seed=5)).cuda()
    out = (torch.empty(10, dtype=torch.int32, device="cuda"), torch.empty(10, dtype=torch.int32, device="cuda"))
    with pytest.raises(mh.MHError) as ei:
        mh.sample_unweighted_noalloc(x, out, seed=2)
    assert ei.value.status == mh.MH_ECAPACITY
