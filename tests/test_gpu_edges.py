"""Canonical order of edge lists (mh_sort_edges) on the GPU, against numpy's
lexsort of the same arrays: sampled edge lists (unweighted and weighted), a
hub whose run of edges exceeds the LDS sort, and small or ragged sizes."""
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


def dev_i32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def check(mh, src, dst, w=None):
    s, d = dev_i32(src), dev_i32(dst)
    ww = None if w is None else dev_i32(w)
    mh.sort_edges(s, d, ww)
    o = np.lexsort((np.asarray(dst), np.asarray(src))) if w is None else np.lexsort(
        (np.asarray(w), np.asarray(dst), np.asarray(src)))
    assert np.array_equal(s.cpu().numpy(), np.asarray(src)[o])
    assert np.array_equal(d.cpu().numpy(), np.asarray(dst)[o])
    if w is not None:
        assert np.array_equal(ww.cpu().numpy(), np.asarray(w)[o])


def test_sampled_edges(mh):
    x = workloads.lognormal_x(np.random.default_rng(3), 200_000, -4, 1.5)
    s, d = mh.sample_unweighted(torch.as_tensor(x).cuda(), seed=2, replica=1)
    assert s.numel() > 10_000
    check(mh, s.cpu().numpy(), d.cpu().numpy())
    # the order is canonical: the same edges in another order sort to the same list
    mh.sort_edges(s, d)
    p = torch.randperm(s.numel(), device=s.device)
    s2, d2 = s[p].contiguous(), d[p].contiguous()
    mh.sort_edges(s2, d2)
    assert torch.equal(s, s2) and torch.equal(d, d2)


def test_sampled_weighted_edges(mh):
    rng = np.random.default_rng(4)
    k = workloads.powerlaw_degrees(rng, 50_000, 2.3, 1, 500)
    s_ = np.round(k * (1 + rng.gamma(2.0, 3.0, k.size)))
    x, y = workloads.uecm_recipe(k, s_)
    src, dst, w = mh.sample_weighted(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(), seed=5)
    check(mh, src.cpu().numpy(), dst.cpu().numpy(), w.cpu().numpy())


def test_hub_beyond_lds_and_ragged_sizes(mh):
    rng = np.random.default_rng(5)
    # one source with 30,000 edges in random order, then short runs
    hub_dst = rng.permutation(40_000)[:30_000]
    src = np.concatenate([np.full(30_000, 7), rng.integers(0, 50_000, 20_000)])
    dst = np.concatenate([hub_dst, rng.integers(0, 50_000, 20_000)])
    p = rng.permutation(src.size)
    check(mh, src[p], dst[p])
    for m in (0, 1, 2, 63, 64, 65, 4097, 70_001):
        a = rng.integers(0, 1 << 31, m, dtype=np.int64)
        b = rng.integers(0, 1 << 31, m, dtype=np.int64)
        check(mh, a, b, rng.integers(1, 1000, m))


def test_runs_of_every_length_up_to_the_wave_limit(mh):
    # sources with 2 to 300 edges each (every length from 2 to 300 several
    # times, in random order): runs up to 64 are sorted by a wave over its
    # lanes, up to 128 and 256 by a wave's register network, longer ones by the
    # block; destinations drawn so that some runs hold equal high bytes
    rng = np.random.default_rng(6)
    lens = np.concatenate([np.arange(2, 301)] * 6)
    rng.shuffle(lens)
    src = np.repeat(np.arange(len(lens)) * 3 + 11, lens)
    dst = np.concatenate([rng.choice(1 << int(rng.integers(9, 31)), size=L, replace=False) for L in lens])
    p = rng.permutation(src.size)
    check(mh, src[p], dst[p])
    # already ordered within runs except for one swapped pair
    src2, dst2 = src.copy(), np.concatenate([np.sort(rng.choice(1 << 20, size=L, replace=False)) for L in lens])
    off = np.concatenate([[0], np.cumsum(lens)])
    for r in range(0, len(lens), 7):
        i = off[r] + int(rng.integers(0, lens[r] - 1))
        dst2[i], dst2[i + 1] = dst2[i + 1], dst2[i]
    check(mh, src2, dst2)
