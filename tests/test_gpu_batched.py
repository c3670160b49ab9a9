"""GPU parity of the batched persistent sampler against the oracle.

Sample (network i, replica r) of a batch must equal the oracle's sample of
network i with the same seed, replica and plan parameter, edge for edge (the
bar of tests/parity.py: counted divergences in the oracle's near-tie rows
only); the degree-sink mode must equal the degree sequences of those samples;
a captured hipGraph replays to the same result as the eager call.  Every
sample of a batch is compared.
"""
import numpy as np
import pytest

import oracle
import parity

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


def _nets(seed, sizes, weighted=False):
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for n in sizes:
        xs.append(np.exp(rng.normal(-3.0, 1.8, n)))
        if weighted:
            ys.append(rng.uniform(0.1, 0.95, n))
    return xs, (ys if weighted else None)


def _keys(src, dst, n, w=None):
    key = np.asarray(src, np.int64) * n + np.asarray(dst, np.int64)
    if w is None:
        return np.sort(key), None
    o = np.lexsort((np.asarray(w), key))
    return key[o], np.asarray(w)[o]


def _compare_sample(src, dst, w, sel, ora, n, label):
    """Edges of one sample of a batch (rows `sel` of the batch's lists) against
    the oracle's sample."""
    return parity.edge_divergences(src[sel], dst[sel], None if w is None else w[sel], ora.src, ora.dst,
                                   ora.w if w is not None else None, n, ora.tie_rows, label=label)


def _compare_degrees(deg, ora, n, label):
    """A degree-sink sequence against the oracle sample's degrees: identical,
    or (near-tie rows only) differing by at most two units per allowed
    divergence."""
    ref = np.bincount(ora.src, minlength=n) + np.bincount(ora.dst, minlength=n)
    if len(ora.tie_rows) == 0:
        assert np.array_equal(deg, ref), label
        return
    assert int(np.abs(deg.astype(np.int64) - ref).sum()) <= 2 * parity.allowed_divergences(len(ora.src)), label


@pytest.mark.parametrize("seg_work", [0, 8])
def test_batch_edges_match_oracle(mh, seg_work):
    sizes = [1, 2, 300, 2500, 40, 1800]
    xs, _ = _nets(1, sizes)
    b = mh.Batch([dev(x) for x in xs], seg_work=seg_work, max_samples=64)
    net = [i for i in range(len(sizes)) for _ in range(3)]
    rep = [r for _ in sizes for r in (0, 5, 9)]
    src, dst, _, sid = b.sample_edges(net, rep, seed=17)
    src, dst, sid = src.cpu().numpy(), dst.cpu().numpy(), sid.cpu().numpy()
    compared = 0
    for s, (i, r) in enumerate(zip(net, rep)):
        ora = oracle.sample_mh(xs[i], None, seed=17, replica=r, seg_work=seg_work)
        _compare_sample(src, dst, None, sid == s, ora, sizes[i], f"batch net {i} replica {r}")
        compared += 1
    assert compared == len(net)


@pytest.mark.parametrize("weighted", [False, True])
def test_batch_edges_labelled_when_lanes_cross_samples(mh, weighted):
    # one block: every lane takes many items in turn, from one sample and then
    # the next, and may accept the last candidate of a segment in the same
    # step that it moves on; each edge keeps the sample it was drawn in
    sizes = [700, 30, 1500, 200, 900]
    xs, ys = _nets(5 if weighted else 4, sizes, weighted=weighted)
    b = mh.Batch([dev(x) for x in xs], [dev(y) for y in ys] if weighted else None, seg_work=4, max_samples=16)
    net = [0, 1, 2, 3, 4, 2, 0]
    rep = [0, 0, 1, 2, 3, 4, 5]
    for grid in (1, 2):
        src, dst, w, sid = b.sample_edges(net, rep, seed=11, grid_blocks=grid)
        src, dst, sid = src.cpu().numpy(), dst.cpu().numpy(), sid.cpu().numpy()
        w = None if w is None else w.cpu().numpy()
        compared = 0
        for s, (i, r) in enumerate(zip(net, rep)):
            ora = oracle.sample_mh(xs[i], ys[i] if weighted else None, seed=11, replica=r, seg_work=4)
            _compare_sample(src, dst, w, sid == s, ora, sizes[i], f"grid {grid} sample {s}")
            compared += 1
        assert compared == len(net)


def test_batch_weighted_edges_match_oracle(mh):
    sizes = [500, 1200, 64]
    xs, ys = _nets(2, sizes, weighted=True)
    b = mh.Batch([dev(x) for x in xs], [dev(y) for y in ys], seg_work=4, max_samples=16)
    net, rep = [0, 1, 2, 1], [0, 0, 3, 7]
    src, dst, w, sid = b.sample_edges(net, rep, seed=3)
    src, dst, w, sid = (t.cpu().numpy() for t in (src, dst, w, sid))
    compared = 0
    for s, (i, r) in enumerate(zip(net, rep)):
        ora = oracle.sample_mh(xs[i], ys[i], seed=3, replica=r, seg_work=4)
        _compare_sample(src, dst, w, sid == s, ora, sizes[i], f"weighted batch sample {s}")
        compared += 1
    assert compared == len(net)


def test_batch_degrees_match_oracle(mh):
    sizes = [700, 3000, 150]
    xs, _ = _nets(3, sizes)
    b = mh.Batch([dev(x) for x in xs], seg_work=16, max_samples=16)
    net, rep = [0, 1, 2, 1, 0], [1, 1, 1, 2, 8]
    deg, off = b.sample_degrees(net, rep, seed=5)
    deg = deg.cpu().numpy()
    for s, (i, r) in enumerate(zip(net, rep)):
        ora = oracle.sample_mh(xs[i], None, seed=5, replica=r, seg_work=16)
        _compare_degrees(deg[off[s]:off[s + 1]], ora, sizes[i], f"degree sink sample {s}")


def test_graph_replays_match_eager(mh):
    sizes = [1500, 400]
    xs, _ = _nets(4, sizes)
    b = mh.Batch([dev(x) for x in xs], seg_work=8, max_samples=8)
    net = torch.tensor([0, 1, 0], dtype=torch.int32, device="cuda")
    rep = torch.tensor([2, 2, 3], dtype=torch.int32, device="cuda")
    eager, off = b.sample_degrees(net.cpu(), rep.cpu(), seed=9)
    eager = eager.cpu().numpy()
    deg = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
    g = b.capture_degrees(net, rep, 9, deg, off.cuda())
    for _ in range(4):
        deg.fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(deg.cpu().numpy(), eager)
        # eager work between replays
        b.sample_degrees([1], [0], seed=1)


def _staged_nets(seed, weighted):
    # a network of three counting windows (70,000 columns), one of two, and
    # small ones; weights kept sparse enough for the oracle
    rng = np.random.default_rng(seed)
    sizes = [70_000, 40_000, 3000, 150]
    xs = [np.exp(rng.normal(-6.0, 1.5, n)) for n in sizes[:2]] + [np.exp(rng.normal(-3.0, 1.8, n)) for n in sizes[2:]]
    ys = [rng.uniform(0.1, 0.95, n) for n in sizes] if weighted else None
    return sizes, xs, ys


@pytest.mark.parametrize("weighted", [False, True])
def test_staged_degrees_equal_atomic_degrees(mh, weighted):
    # the slot-buffer degree sink gives the atomic sink's degrees at any slot
    # capacity: none (no room for the regions' bookkeeping: every column by
    # atomics), a few thousand (regions cut, the rest by atomics) and ample;
    # the atomic sink equals the oracle
    sizes, xs, ys = _staged_nets(12, weighted)
    b = mh.Batch([dev(x) for x in xs], [dev(y) for y in ys] if weighted else None, seg_work=16, max_samples=16)
    net, rep = [0, 1, 2, 3, 0, 2, 1], [0, 0, 1, 2, 5, 3, 9]
    ref, off = b.sample_degrees(net, rep, seed=7)
    ref = ref.cpu().numpy()
    for s in (0, 2):
        i, r = net[s], rep[s]
        ora = oracle.sample_mh(xs[i], ys[i] if weighted else None, seed=7, replica=r, seg_work=16)
        _compare_degrees(ref[off[s]:off[s + 1]], ora, sizes[i], f"atomic sink sample {s}")
    for cap in (0, 5000, 1 << 22):
        slots = torch.empty(cap, dtype=torch.int32, device="cuda")
        deg, off2 = b.sample_degrees(net, rep, seed=7, slots=slots)
        assert np.array_equal(off2.numpy(), off.numpy())
        assert np.array_equal(deg.cpu().numpy(), ref), f"staged sink, {cap} slots"
    # a smaller batch after a larger one reuses the cursors and regions
    slots = torch.empty(1 << 22, dtype=torch.int32, device="cuda")
    deg, off3 = b.sample_degrees([3, 0], [2, 5], seed=7, slots=slots)
    deg = deg.cpu().numpy()
    assert np.array_equal(deg[off3[0]:off3[1]], ref[off[3]:off[4]])
    assert np.array_equal(deg[off3[1]:off3[2]], ref[off[4]:off[5]])


def test_staged_degrees_at_the_window_limits(mh):
    # 128 windows of 2^15 ids (4,194,304 nodes): one bin per sample, so the
    # flushes that hold several samples add all but the lowest by atomics;
    # one node more (129 windows): the call counts by atomics throughout.
    # Sparse x (about 1e5 edges a sample); the staged degrees must equal the
    # atomic sink's exactly.
    rng = np.random.default_rng(15)
    for n_big in (128 << 15, (128 << 15) + 1):
        xs = [np.exp(rng.normal(-9.0, 1.0, n_big)), np.exp(rng.normal(-3.0, 1.8, 2000))]
        b = mh.Batch([dev(x) for x in xs], seg_work=16, max_samples=8)
        net, rep = [0, 1, 0, 1, 1], [0, 0, 1, 1, 2]
        ref, off = b.sample_degrees(net, rep, seed=3)
        slots = torch.empty(1 << 24, dtype=torch.int32, device="cuda")
        deg, _ = b.sample_degrees(net, rep, seed=3, slots=slots)
        assert np.array_equal(deg.cpu().numpy(), ref.cpu().numpy()), f"{n_big} nodes"
        assert int(ref.sum()) > 0
        del b, slots, deg, ref


@pytest.mark.parametrize("grid", [1, 3, 0])
def test_staged_degrees_many_samples_per_flush(mh, grid):
    # 120 samples, the largest network of three windows (42 samples a flush
    # can bin): on one block a wave's flushes hold pairs of samples far apart
    # (added by atomics) as well as near ones (binned); staged and atomic
    # sinks must agree exactly at every grid
    sizes, xs, _ = _staged_nets(16, False)
    b = mh.Batch([dev(x) for x in xs], seg_work=8, max_samples=128)
    rng = np.random.default_rng(17)
    net = rng.integers(0, len(xs), 120).tolist()
    rep = rng.integers(0, 1000, 120).tolist()
    ref, off = b.sample_degrees(net, rep, seed=4, grid_blocks=grid)
    slots = torch.empty(1 << 24, dtype=torch.int32, device="cuda")
    deg, _ = b.sample_degrees(net, rep, seed=4, grid_blocks=grid, slots=slots)
    assert np.array_equal(deg.cpu().numpy(), ref.cpu().numpy()), f"grid {grid}"


def test_staged_degree_graph_replays_match_eager(mh):
    sizes, xs, _ = _staged_nets(13, False)
    b = mh.Batch([dev(x) for x in xs], seg_work=8, max_samples=8)
    net = torch.tensor([0, 3, 1], dtype=torch.int32, device="cuda")
    rep = torch.tensor([2, 2, 3], dtype=torch.int32, device="cuda")
    eager, off = b.sample_degrees(net.cpu(), rep.cpu(), seed=9)
    eager = eager.cpu().numpy()
    slots = torch.empty(1 << 21, dtype=torch.int32, device="cuda")
    deg = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
    g = b.capture_degrees(net, rep, 9, deg, off.cuda(), slots=slots)
    for _ in range(3):
        deg.fill_(-1)
        slots.fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(deg.cpu().numpy(), eager)
        b.sample_degrees([2], [0], seed=1, slots=slots)


def test_staged_degrees_reject_bad_slots(mh):
    _, xs, _ = _staged_nets(14, False)
    b = mh.Batch([dev(xs[3])], seg_work=8, max_samples=4)
    with pytest.raises(ValueError):
        b.sample_degrees([0], [0], slots=torch.empty(10, dtype=torch.int64, device="cuda"))


def test_graph_edge_replays_match_eager(mh):
    xs, _ = _nets(5, [2000])
    b = mh.Batch([dev(xs[0])], seg_work=16, max_samples=4)
    net = torch.tensor([0, 0], dtype=torch.int32, device="cuda")
    rep = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    s0, d0, _, sid0 = b.sample_edges(net.cpu(), rep.cpu(), seed=2)
    k0 = np.sort(sid0.cpu().numpy().astype(np.int64) * 2**40 + s0.cpu().numpy().astype(np.int64) * 2000 +
                 d0.cpu().numpy())
    cap = len(s0) + mh.BATCH_EDGE_SLACK
    src = torch.empty(cap, dtype=torch.int32, device="cuda")
    dst = torch.empty(cap, dtype=torch.int32, device="cuda")
    sid = torch.empty(cap, dtype=torch.int32, device="cuda")
    g = b.capture_edges(net, rep, 2, src, dst, None, sid, cap)
    for _ in range(3):
        g.launch()
        m = b.result(cap)
        assert m == len(s0)
        k = np.sort(sid[:m].cpu().numpy().astype(np.int64) * 2**40 + src[:m].cpu().numpy().astype(np.int64) * 2000 +
                    dst[:m].cpu().numpy())
        assert np.array_equal(k, k0)


def test_edge_output_room_for_chunks(mh):
    # each wave reserves its output 4096 slots at a time: at the exact edge
    # count the call reports a capacity that suffices; the retry (the
    # binding's) gives the same edges, and so do grids of one and three blocks
    xs, _ = _nets(9, [3000, 1500, 700])
    b = mh.Batch([dev(x) for x in xs], seg_work=8, max_samples=8)
    net, rep = [0, 1, 2, 0], [0, 0, 1, 1]
    s0, d0, _, sid0 = b.sample_edges(net, rep, seed=3)
    n = len(s0)

    def key(s, d, sid):
        return np.sort(sid.cpu().numpy().astype(np.int64) * 2**40 + s.cpu().numpy().astype(np.int64) * 4096 +
                       d.cpu().numpy())

    k0 = key(s0, d0, sid0)
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    b.sample_edges_async(torch.tensor(net, dtype=torch.int32, device="cuda"),
                         torch.tensor(rep, dtype=torch.int32, device="cuda"), 3, bufs[0], bufs[1], None, bufs[2], n)
    m = b.result(n)
    assert m == n or -m > n  # not enough room for the chunks: a larger capacity is reported
    s1, d1, _, sid1 = b.sample_edges(net, rep, seed=3, capacity=n)
    assert np.array_equal(key(s1, d1, sid1), k0)
    for grid in (1, 3):
        s2, d2, _, sid2 = b.sample_edges(net, rep, seed=3, grid_blocks=grid)
        assert np.array_equal(key(s2, d2, sid2), k0)
    for i, (nn, r) in enumerate(zip(net, rep)):
        ora = oracle.sample_mh(xs[nn], None, seed=3, replica=r, seg_work=8)
        sel = sid0.cpu().numpy() == i
        _compare_sample(s0.cpu().numpy(), d0.cpu().numpy(), None, sel, ora, len(xs[nn]), f"chunked sample {i}")


def test_autotune_then_parity(mh):
    sizes = [2000, 900, 4000]
    xs, _ = _nets(6, sizes)
    b = mh.Batch([dev(x) for x in xs], seg_work=32, max_samples=16)
    best = b.autotune([0, 1, 2], [0, 0, 0], seg_candidates=(4, 16, 64), grid_candidates=(0, 64))
    assert best["seg_work"] in (4, 16, 64) and best["ms"] > 0
    src, dst, _, sid = b.sample_edges([2], [4], seed=8)
    ora = oracle.sample_mh(xs[2], None, seed=8, replica=4, seg_work=best["seg_work"])
    src, dst = src.cpu().numpy(), dst.cpu().numpy()
    _compare_sample(src, dst, None, np.ones(len(src), bool), ora, 4000, "autotuned batch")


def test_bad_network_index(mh):
    xs, _ = _nets(7, [100])
    b = mh.Batch([dev(xs[0])], max_samples=4)
    with pytest.raises(mh.MHError):
        b.sample_degrees([3], [0])
    # the error belongs to that call: the next call on the batch succeeds
    deg, off = b.sample_degrees([0], [0], seed=2)
    ora = oracle.sample_mh(xs[0], None, seed=2, replica=0, seg_work=mh.DEFAULT_SEG_WORK)
    _compare_degrees(deg.cpu().numpy(), ora, 100, "after a failed call")
    # the same through the slot buffer: a bad index among good ones fails the
    # call, and the next staged call counts as the atomic one did
    slots = torch.empty(1 << 16, dtype=torch.int32, device="cuda")
    with pytest.raises(mh.MHError):
        b.sample_degrees([0, 3, 0], [0, 0, 1], slots=slots)
    deg2, _ = b.sample_degrees([0], [0], seed=2, slots=slots)
    assert np.array_equal(deg2.cpu().numpy(), deg.cpu().numpy())


def test_batch_largest_ensemble_networks_match_oracle(mh):
    # the three largest networks of the 256-network ensemble (N near 2e5,
    # x = exp(Normal(-5, 2)), ~3e7 edges a sample) at the segment length the
    # ensemble's autotuner picks on the bench (32), default grid: every sample
    # edge for edge, and its degree-sink sequence
    import workloads

    nets = workloads.cfg4_networks(seed=4)
    big = sorted(range(len(nets)), key=lambda i: -len(nets[i].x))[:3]
    xs = [nets[i].x for i in big]
    assert min(len(x) for x in xs) >= 100_000
    b = mh.Batch([dev(x) for x in xs], seg_work=32, max_samples=8)
    net, rep = [0, 1, 2], [0, 7, 15]
    ora = [oracle.sample_mh(xs[i], None, seed=1, replica=r, seg_work=32, capacity=40_000_000)
           for i, r in zip(net, rep)]
    cap = sum(o.n_edges for o in ora) + (1 << 20)
    src, dst, _, sid = b.sample_edges(net, rep, seed=1, capacity=cap)
    src, dst, sid = src.cpu().numpy(), dst.cpu().numpy(), sid.cpu().numpy()
    for s, (i, r) in enumerate(zip(net, rep)):
        _compare_sample(src, dst, None, sid == s, ora[s], len(xs[i]), f"ensemble network {big[i]} replica {r}")
    del src, dst, sid
    deg, off = b.sample_degrees(net, rep, seed=1)
    deg = deg.cpu().numpy()
    for s, (i, r) in enumerate(zip(net, rep)):
        _compare_degrees(deg[off[s]:off[s + 1]], ora[s], len(xs[i]), f"ensemble degrees {big[i]} replica {r}")
    # the staged sink on the same samples (seven windows each): the atomic sink's degrees
    slots = torch.empty(200_000_000, dtype=torch.int32, device="cuda")
    sdeg, _ = b.sample_degrees(net, rep, seed=1, slots=slots)
    assert np.array_equal(sdeg.cpu().numpy(), deg)
