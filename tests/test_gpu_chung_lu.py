"""GPU parity of the Chung-Lu comparison model and of the bias statistics
(Sec. 2.1, Fig. 1; Sec. 2.3) against the CPU oracle, through the C-ABI:
Chung-Lu edge lists (tests/parity.py's bar), counts by rank of UBCM and
Chung-Lu samples (the rich-club numerators), triangle counts (exact), and the
bias itself on a Holme-Kim network's degrees."""
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


def dev_i32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _cl_weights(seed, n, kmax=3000):
    # w = k / sqrt(2M) for power-law degrees: the hubs' products exceed 1
    k = workloads.powerlaw_degrees(np.random.default_rng(seed), n, 2.1, 2, kmax).astype(np.float64)
    return k / np.sqrt(k.sum())


def _fit_ubcm_cpu(k, tol=1e-10):
    kc, inv, cnt = np.unique(np.asarray(k, np.float64), return_inverse=True, return_counts=True)
    x = kc / np.sqrt(np.sum(k))
    for _ in range(20_000):
        kk, _ = oracle.expected_degree(x, None, cnt.astype(np.float64))
        if np.max(np.abs(kk - kc) / kc) <= tol:
            break
        x = x * (kc / kk)
    return x[inv.reshape(-1)]


@pytest.mark.parametrize("seg_work", [0, 1, 4, 32])
def test_chung_lu_edges_match_oracle(mh, seg_work):
    w = _cl_weights(1, 4000)
    top = np.sort(w)[::-1][:50]
    assert (np.outer(top, top) > 1).sum() > 100  # a dense core where q = 1
    for replica in (0, 3):
        src, dst, st = mh.sample_chung_lu(dev(w), seed=13, replica=replica, seg_work=seg_work, stats=True)
        ora = oracle.sample_chung_lu(w, seed=13, replica=replica, seg_work=seg_work)
        parity.edge_divergences(src.cpu().numpy(), dst.cpu().numpy(), None, ora.src, ora.dst, None, len(w),
                                ora.tie_rows, label=f"chung-lu seg {seg_work} replica {replica}")
        if len(ora.tie_rows) == 0:
            for key in ("steps", "proposals", "accepts", "segments"):
                assert st[key] == ora.stats[key], key


def test_chung_lu_full_size_matches_oracle(mh):
    # N = 1,000,000 power-law degrees (2.1 on [1, 10^4]), w = k / sqrt(2M): the
    # Chung-Lu twin of the N = 1M workload, timed configuration (seg_work 8)
    k = workloads.cfg2_degrees().astype(np.float64)
    w = k / np.sqrt(k.sum())
    src, dst = mh.sample_chung_lu(dev(w), seed=1, replica=1000, seg_work=8)
    ora = oracle.sample_chung_lu(w, seed=1, replica=1000, seg_work=8, capacity=3_000_000)
    parity.edge_divergences(src.cpu().numpy(), dst.cpu().numpy(), None, ora.src, ora.dst, None, len(w),
                            ora.tie_rows, label="chung-lu N=1M")


def test_chung_lu_edge_cases(mh):
    for w in (np.array([0.5]), np.array([2.0, 3.0]), np.zeros(50), np.full(300, 1.5), np.full(300, 0.05)):
        src, dst = mh.sample_chung_lu(dev(w), seed=2, seg_work=4)
        ora = oracle.sample_chung_lu(w, seed=2, seg_work=4)
        parity.edge_divergences(src.cpu().numpy(), dst.cpu().numpy(), None, ora.src, ora.dst, None, len(w),
                                ora.tie_rows, label=f"chung-lu edge case n={len(w)}")
    with pytest.raises(mh.MHError) as ei:
        mh.sample_chung_lu(dev(np.array([1.0, np.nan])))
    assert ei.value.status == mh.MH_EINVAL


@pytest.mark.parametrize("model", ["ubcm", "chung_lu"])
def test_rank_counts_match_oracle(mh, model):
    # counts by rank of the larger endpoint, computed in the sweep without an
    # edge list, against the oracle sample's edges mapped to ranks
    w = _cl_weights(2, 6000)
    mcode = mh.MH_MODEL_CHUNG_LU if model == "chung_lu" else mh.MH_MODEL_UBCM
    for replica in (0, 1):
        cnt, m = mh.rank_counts(dev(w), model=mcode, seed=4, replica=replica, seg_work=8)
        cnt = cnt.cpu().numpy().astype(np.int64)
        ora = (oracle.sample_chung_lu if model == "chung_lu" else
               lambda *a, **kw: oracle.sample_mh(a[0], None, **kw))(w, seed=4, replica=replica, seg_work=8)
        ref = oracle.rank_counts(ora.src, ora.dst, oracle.order(w))
        if len(ora.tie_rows) == 0:
            assert np.array_equal(cnt, ref)
            assert m == ora.n_edges
        else:
            assert int(np.abs(cnt - ref).sum()) <= 2 * parity.allowed_divergences(ora.n_edges)
        # the same sample as the edge-list call
        sampler = mh.sample_chung_lu if model == "chung_lu" else mh.sample_unweighted
        s, d = sampler(dev(w), seed=4, replica=replica, seg_work=8)
        perm = mh.order(dev(w))[0].cpu().numpy()
        assert np.array_equal(cnt, oracle.rank_counts(s.cpu().numpy(), d.cpu().numpy(), perm))


def test_triangles_match_oracle(mh):
    # the Holme-Kim network, sampled networks of both models, a complete graph
    s, d = workloads.holme_kim()
    assert mh.count_triangles(dev_i32(s), dev_i32(d), 5000) == oracle.count_triangles(s, d, 5000)
    assert mh.count_triangles(dev_i32(d), dev_i32(s), 5000) == oracle.count_triangles(s, d, 5000)
    w = _cl_weights(3, 20_000, kmax=2000)
    for sampler in (mh.sample_chung_lu, mh.sample_unweighted):
        src, dst = sampler(dev(w), seed=6, replica=2)
        t = mh.count_triangles(src, dst, len(w))
        assert t == oracle.count_triangles(src.cpu().numpy(), dst.cpu().numpy(), len(w))
        assert t > 0
    n = 200
    iu = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
    assert mh.count_triangles(dev_i32(iu[:, 1]), dev_i32(iu[:, 0]), n) == n * (n - 1) * (n - 2) // 6
    assert mh.count_triangles(dev_i32(np.zeros(0)), dev_i32(np.zeros(0)), 10) == 0
    for bad in ((np.array([0, 1]), np.array([1, 1])), (np.array([0, 5]), np.array([1, 2]))):
        with pytest.raises(mh.MHError) as ei:
            mh.count_triangles(dev_i32(bad[0]), dev_i32(bad[1]), 5)
        assert ei.value.status == mh.MH_EINVAL


def test_chung_lu_bias_on_holme_kim_degrees(mh):
    # Sec. 2.1 / Fig. 1 on the Holme-Kim network's degrees: the Chung-Lu model
    # puts more edges among the top-degree nodes and more triangles than the
    # unbiased model fitted to the same degrees
    s, d = workloads.holme_kim()
    n = 5000
    k = (np.bincount(s, minlength=n) + np.bincount(d, minlength=n)).astype(np.float64)
    w = k / np.sqrt(k.sum())
    x = _fit_ubcm_cpu(k)
    R = 20
    top = int(0.01 * n)
    rich = {"cl": [], "ubcm": []}
    tri = {"cl": [], "ubcm": []}
    for r in range(R):
        for name, sampler, par, model in (("cl", mh.sample_chung_lu, w, mh.MH_MODEL_CHUNG_LU),
                                          ("ubcm", mh.sample_unweighted, x, mh.MH_MODEL_UBCM)):
            cnt, _ = mh.rank_counts(dev(par), model=model, seed=9, replica=r)
            rich[name].append(cnt[:top].sum().item() / (top * (top - 1) / 2))
            src, dst = sampler(dev(par), seed=9, replica=r)
            tri[name].append(mh.count_triangles(src, dst, n))
    assert np.mean(rich["cl"]) > np.mean(rich["ubcm"]) + 3 * np.std(rich["ubcm"]) / np.sqrt(R)
    assert np.mean(tri["cl"]) > np.mean(tri["ubcm"]) + 3 * np.std(tri["ubcm"]) / np.sqrt(R)
    # the unbiased model keeps the expected degrees: its mean edge count is sum(k) / 2
    assert abs(np.mean([c for c in [mh.rank_counts(dev(x), seed=3, replica=r)[1] for r in range(R)]]) - k.sum() / 2) \
        < 4 * np.sqrt(k.sum() / 2 / R)
