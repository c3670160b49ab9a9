"""GPU parity of the bipartite / directed sampler (Sec. 2.6) against the CPU
oracle, through the C-ABI.  Same bar as the one-set sampler (tests/parity.py):
identical edge lists and weights but for counted divergences in the rows of the
oracle's near-tie trace, and identical counters when the trace is empty."""
import numpy as np
import pytest

import oracle
import parity
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def keys(src, dst, nc, w=None):
    k = np.asarray(src, dtype=np.int64) * nc + np.asarray(dst, dtype=np.int64)
    if w is None:
        return np.sort(k), None
    o = np.lexsort((np.asarray(w), k))
    return k[o], np.asarray(w)[o]


def compare(res, ora, nc, weighted=False, label="bipartite"):
    gs, gd = res.src.cpu().numpy(), res.dst.cpu().numpy()
    gw = res.w.cpu().numpy() if weighted else None
    n_div = parity.edge_divergences(gs, gd, gw, ora.src, ora.dst, ora.w if weighted else None, nc, ora.tie_rows,
                                    label=label)
    if len(ora.tie_rows) == 0 and res.stats is not None:
        for k in ("steps", "proposals", "accepts", "segments", "saturated_w"):
            assert res.stats[k] == ora.stats[k], k
    return n_div


def run(mh, xr, xc, yr=None, yc=None, exclude_self=False, seed=1, replica=0, seg_work=16, **kw):
    res = mh.sample_bipartite(dev(xr), dev(xc), None if yr is None else dev(yr), None if yc is None else dev(yc),
                              exclude_self=exclude_self, seed=seed, replica=replica, seg_work=seg_work, stats=True,
                              **kw)
    ora = oracle.sample_bipartite(xr, xc, yr, yc, exclude_self=exclude_self, seed=seed, replica=replica,
                                  seg_work=seg_work)
    compare(res, ora, len(xc), weighted=yr is not None)
    return res, ora


@pytest.mark.parametrize("seg_work", [0, 1, 4, 16, 64])
def test_unweighted_small(mh, seg_work):
    xr, xc, _, _ = workloads.bipartite_params(seed=11, n_rows=3001, n_cols=4700)
    for replica in (0, 1):
        run(mh, xr, xc, seed=5, replica=replica, seg_work=seg_work)


@pytest.mark.parametrize("seg_work", [0, 2, 16])
def test_weighted_small(mh, seg_work):
    xr, xc, yr, yc = workloads.bipartite_params(seed=12, n_rows=2500, n_cols=1800, weighted=True)
    res, ora = run(mh, xr, xc, yr, yc, seed=6, replica=2, seg_work=seg_work)
    assert ora.n_edges > 1000


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("seg_work", [0, 16])
def test_directed_small(mh, weighted, seg_work):
    xo, xi, yo, yi = workloads.directed_params(seed=13, n=4000, weighted=weighted)
    res, ora = run(mh, xo, xi, yo, yi, exclude_self=True, seed=7, replica=1, seg_work=seg_work)
    assert not np.any(res.src.cpu().numpy() == res.dst.cpu().numpy())
    # without the flag the same call may contain self-pairs and has as many candidates
    res2, ora2 = run(mh, xo, xi, yo, yi, exclude_self=False, seed=7, replica=1, seg_work=seg_work)
    assert ora2.stats["proposals"] == ora.stats["proposals"]


def test_dense_hubs_overflow_records(mh):
    # 20 rows with p ~ 1/2 against 60k columns: ~15k segments per row at
    # seg_work 4, far more heavy items than stored records (rows + 4096), so the
    # sweep locates most segments itself.
    rng = np.random.default_rng(14)
    xr = np.full(20, 1.0) * rng.uniform(0.5, 2.0, 20)
    xc = rng.uniform(0.3, 3.0, 60_000)
    run(mh, xr, xc, seed=8, seg_work=4)
    yr = rng.uniform(0.1, 0.6, 20)
    yc = rng.uniform(0.1, 0.9, 60_000)
    run(mh, xr / yr, xc / yc, yr, yc, seed=9, seg_work=4)


def test_edge_cases(mh):
    one = np.array([1.5])
    cases = [
        (one, one), (one, np.array([0.0, 2.0, 0.5])), (np.zeros(50), np.full(30, 0.4)),
        (np.full(300, 0.2), np.zeros(70)), (np.full(257, 0.3), np.full(129, 0.3)),
    ]
    for xr, xc in cases:
        for seg_work in (0, 1, 16):
            run(mh, xr, xc, seed=3, seg_work=seg_work)
    res, _ = run(mh, np.full(100, 0.5), np.full(100, 0.5), exclude_self=True, seed=3)
    # empty sets: empty sample
    for nr, nc in ((0, 10), (10, 0), (0, 0)):
        r = mh.sample_bipartite(dev(np.full(nr, 0.5)), dev(np.full(nc, 0.5)), stats=True)
        assert r.src.numel() == 0 and r.stats["proposals"] == 0
    # only products across the sets must be finite: z+ = 1e160 is fine against small z-
    run(mh, np.array([1e160, 1.0, 0.0]), np.array([1e-160, 0.5, 2e-161]), seed=5)
    # y+ alone may exceed 1 when every product y+ y- stays below 1
    run(mh, np.full(40, 0.5), np.full(60, 0.5), np.full(40, 1.5), np.full(60, 0.6), seed=4)


def test_capacity_retry_is_identical(mh):
    xr, xc, _, _ = workloads.bipartite_params(seed=15, n_rows=2000, n_cols=2000)
    full = mh.sample_bipartite(dev(xr), dev(xc), seed=9)
    small = mh.sample_bipartite(dev(xr), dev(xc), seed=9, capacity=max(1, full.src.numel() // 3))
    assert np.array_equal(keys(full.src.cpu().numpy(), full.dst.cpu().numpy(), 2000)[0],
                          keys(small.src.cpu().numpy(), small.dst.cpu().numpy(), 2000)[0])


@pytest.mark.parametrize("bad", ["nan_row", "neg_col", "inf_col", "overflow", "y"])
def test_invalid_parameters(mh, bad):
    xr, xc = np.full(100, 0.1), np.full(80, 0.1)
    yr, yc = np.full(100, 0.5), np.full(80, 0.5)
    if bad == "nan_row":
        xr[7] = np.nan
    elif bad == "neg_col":
        xc[3] = -1.0
    elif bad == "inf_col":
        xc[0] = np.inf
    elif bad == "overflow":
        xr[5], xc[9] = 1e160, 1e160  # largest row z times largest column z overflows
    with pytest.raises(mh.MHError) as ei:
        if bad == "y":
            yr[4], yc[2] = 1.1, 0.95
            mh.sample_bipartite(dev(xr), dev(xc), dev(yr), dev(yc))
        else:
            mh.sample_bipartite(dev(xr), dev(xc))
    assert ei.value.status == mh.MH_EINVAL


def test_full_size_bipartite(mh):
    # 1,000,000 rows (degrees power law 2.1) x 500,000 columns (2.5), the
    # default segment size
    xr, xc, _, _ = workloads.bipartite_params()
    res = mh.sample_bipartite(dev(xr), dev(xc), seed=1, replica=3, seg_work=8, stats=True)
    ora = oracle.sample_bipartite(xr, xc, seed=1, replica=3, seg_work=8, capacity=6_000_000)
    compare(res, ora, len(xc))


def test_full_size_directed_weighted(mh):
    xo, xi, yo, yi = workloads.directed_params(n=300_000, weighted=True)
    res = mh.sample_bipartite(dev(xo), dev(xi), dev(yo), dev(yi), exclude_self=True, seed=2, replica=0,
                              seg_work=16, stats=True)
    ora = oracle.sample_bipartite(xo, xi, yo, yi, exclude_self=True, seed=2, replica=0, seg_work=16,
                                  capacity=4_000_000)
    compare(res, ora, len(xi), weighted=True)
