"""Pins of the oracle's bipartite / directed sampler (Sec. 2.6).

The exact law is the bipartite brute-force model: every (row i, column j) pair
is an edge independently with probability p_ij = t/(1+t), t = x+_i x-_j
(unweighted), or t/(1 - y+_i y-_j + t), t = z+_i z-_j (weighted, geometric
weight with ratio y+_i y-_j).  The directed model is the same with rows = out
parameters, columns = in parameters and the pairs i == j left out.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enumerate as en


def _p_bip(xr, xc, yr=None, yc=None):
    if yr is None:
        t = np.outer(xr, xc)
        return t / (1.0 + t), None
    t = np.outer(xr * yr, xc * yc)
    b = np.outer(yr, yc)
    return t / (1.0 - b + t), b


def _order(z):
    return np.lexsort((np.arange(len(z)), -z))


def _row_law_bip(zrs_r, zcs, segments, yr_r=None, ycs=None, Y=None):
    """Exact law of one row's accepted columns: chains over the given column
    segments, each starting with the proposal probability of its first column."""
    p, q = {}, {}
    for j in range(len(zcs)):
        t = zrs_r * zcs[j]
        if ycs is None:
            p[j] = en.ubcm_p(t)
            q[j] = p[j]
        else:
            p[j] = en.uecm_p(t, yr_r * ycs[j])
            q[j] = en.uecm_bound(t, Y)
    law = {frozenset(): en.Fraction(1)}
    for a, b in segments:
        law = en.combine(law, en.segment_law(p, q, a, b, q[a]))
    return law, en.bernoulli_law(p, list(range(len(zcs))))


@pytest.mark.parametrize("seg_work", [0, 1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_bipartite_rows_exact(seg_work, weighted):
    rng = np.random.default_rng(100 + seg_work + 10 * weighted)
    nr, nc = 3, 6
    xr = np.exp(rng.normal(0.0, 1.0, nr))
    xc = np.exp(rng.normal(0.0, 1.0, nc))
    yr = rng.uniform(0.1, 0.9, nr) if weighted else None
    yc = rng.uniform(0.1, 0.9, nc) if weighted else None
    zr = xr * yr if weighted else xr
    zc = xc * yc if weighted else xc
    pc = _order(zc)
    zcs = zc[pc]
    ycs = yc[pc] if weighted else None
    for i in range(nr):
        Y = yr[i] * yc.max() if weighted else None
        c = 1.0 - Y if weighted else 1.0
        a, b = oracle.plan_row_bipartite(zcs, zr[i], c, seg_work)
        law, target = _row_law_bip(zr[i], zcs, [(int(u), int(v)) for u, v in zip(a, b)], yr[i] if weighted else None, ycs, Y)
        assert law == target


def test_bipartite_bound_from_smallest_column_y_is_biased():
    # Negative control: the row bound Y_r = y_r * min(y-) is not a bound on
    # every column's probability; the chain's law then differs from the target.
    rng = np.random.default_rng(7)
    nc = 5
    xc = np.exp(rng.normal(0.5, 0.5, nc))
    yc = np.array([0.1, 0.2, 0.5, 0.8, 0.9])
    zc = xc * yc
    pc = _order(zc)
    zcs, ycs = zc[pc], yc[pc]
    yr, zr = 0.9, 2.0
    law, target = _row_law_bip(zr, zcs, [(0, nc)], yr, ycs, yr * yc.min())
    assert law != target


def _joint_chi2(samples_fn, pairs, p, R):
    idx = {pr: k for k, pr in enumerate(pairs)}
    ncell = 2 ** len(pairs)
    counts = np.zeros(ncell)
    for rep in range(R):
        src, dst = samples_fn(rep)
        code = 0
        for a, b in zip(src, dst):
            code |= 1 << idx[(int(a), int(b))]
        counts[code] += 1
    probs = np.ones(ncell)
    for k, (i, j) in enumerate(pairs):
        bit = (np.arange(ncell) >> k) & 1
        probs *= np.where(bit == 1, p[i, j], 1.0 - p[i, j])
    exp = probs * R
    keep = exp >= 5
    chi = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    rest_o, rest_e = counts[~keep].sum(), exp[~keep].sum()
    dof = keep.sum() - 1
    if rest_e > 0:
        chi += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    return stats.chi2.sf(chi, dof)


@pytest.mark.parametrize("seg_work", [0, 1])
def test_bipartite_joint_law_chi2(seg_work):
    rng = np.random.default_rng(120 + seg_work)
    nr, nc = 2, 3
    xr = np.exp(rng.normal(-0.2, 1.0, nr))
    xc = np.exp(rng.normal(-0.2, 1.0, nc))
    p, _ = _p_bip(xr, xc)
    pairs = [(i, j) for i in range(nr) for j in range(nc)]

    def fn(rep):
        s = oracle.sample_bipartite(xr, xc, seed=41, replica=rep, seg_work=seg_work, capacity=64)
        return s.src, s.dst

    assert _joint_chi2(fn, pairs, p, 30_000) > 1e-6


@pytest.mark.parametrize("seg_work", [0, 1])
def test_bipartite_weighted_joint_law_and_weights(seg_work):
    rng = np.random.default_rng(130 + seg_work)
    nr, nc = 2, 3
    xr = np.exp(rng.normal(0.5, 1.0, nr))
    xc = np.exp(rng.normal(0.5, 1.0, nc))
    yr = rng.uniform(0.2, 0.9, nr)
    yc = rng.uniform(0.2, 0.9, nc)
    p, b = _p_bip(xr, xc, yr, yc)
    pairs = [(i, j) for i in range(nr) for j in range(nc)]
    W = {}

    def fn(rep):
        s = oracle.sample_bipartite(xr, xc, yr, yc, seed=42, replica=rep, seg_work=seg_work, capacity=64)
        for a, c, w in zip(s.src, s.dst, s.w):
            W.setdefault((int(a), int(c)), []).append(int(w))
        return s.src, s.dst

    assert _joint_chi2(fn, pairs, p, 30_000) > 1e-6
    for (i, j), ws in W.items():
        ws = np.array(ws)
        kmax = 8
        obs = np.array([np.sum(ws == k) for k in range(1, kmax)] + [np.sum(ws >= kmax)], dtype=float)
        pk = np.array([b[i, j] ** (k - 1) * (1 - b[i, j]) for k in range(1, kmax)] + [b[i, j] ** (kmax - 1)])
        e = pk * len(ws)
        keep = e >= 5
        chi = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum()
        assert stats.chi2.sf(chi, max(keep.sum() - 1, 1)) > 1e-6


@pytest.mark.parametrize("weighted", [False, True])
def test_directed_joint_law_no_self_loops(weighted):
    rng = np.random.default_rng(140 + weighted)
    n = 3
    xo = np.exp(rng.normal(0.3, 1.0, n))
    xi = np.exp(rng.normal(0.3, 1.0, n))
    yo = rng.uniform(0.2, 0.9, n) if weighted else None
    yi = rng.uniform(0.2, 0.9, n) if weighted else None
    p, _ = _p_bip(xo, xi, yo, yi)
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j]

    def fn(rep):
        s = oracle.sample_bipartite(xo, xi, yo, yi, exclude_self=True, seed=43, replica=rep, capacity=64)
        assert np.all(s.src != s.dst)
        return s.src, s.dst

    assert _joint_chi2(fn, pairs, p, 30_000) > 1e-6


def test_bipartite_proposal_count_matches_exact_law():
    # Mean number of candidates per sample against the exact path law: pins
    # the chain start (column a's own probability) and the weighted row bound
    # y_r * max(y-) (a looser or tighter bound changes the count).
    rng = np.random.default_rng(150)
    nc = 6
    xc = np.exp(rng.normal(0.0, 1.0, nc))
    yc = rng.uniform(0.3, 0.95, nc)
    xr = np.array([1.7])
    yr = np.array([0.8])
    zc = xc * yc
    pc = _order(zc)
    zcs, ycs = zc[pc], yc[pc]
    zr = float(xr[0] * yr[0])
    Y = float(yr[0] * yc.max())
    p = {j: en.uecm_p(zr * zcs[j], yr[0] * ycs[j]) for j in range(nc)}
    q = {j: en.uecm_bound(zr * zcs[j], Y) for j in range(nc)}
    law = en.segment_proposals(p, q, 0, nc, q[0])
    m1 = float(sum(k * w for k, w in law.items()))
    m2 = float(sum(k * k * w for k, w in law.items()))
    R = 20_000
    props = [oracle.sample_bipartite(xr, xc, yr, yc, seed=13, replica=rep, capacity=64).stats["proposals"]
             for rep in range(R)]
    assert abs(np.mean(props) - m1) <= 4 * np.sqrt((m2 - m1 * m1) / R)


@pytest.mark.parametrize("seg_work", [0, 3, 64])
def test_bipartite_pair_marginals(seg_work):
    rng = np.random.default_rng(160 + seg_work)
    nr, nc = 30, 50
    xr = np.exp(rng.normal(-1.0, 1.2, nr))
    xc = np.exp(rng.normal(-1.0, 1.2, nc))
    p, _ = _p_bip(xr, xc)
    R = 300
    cnt = np.zeros((nr, nc))
    for rep in range(R):
        s = oracle.sample_bipartite(xr, xc, seed=14, replica=rep, seg_work=seg_work)
        np.add.at(cnt, (s.src, s.dst), 1)
    ok = p * R > 5
    z = (cnt / R - p) / np.sqrt(np.maximum(p * (1 - p), 1e-300) / R)
    assert stats.chi2.sf((z[ok] ** 2).sum(), ok.sum()) > 1e-6


def test_bipartite_bf_marginals_and_directed_bf():
    rng = np.random.default_rng(170)
    nr, nc = 20, 25
    xr = np.exp(rng.normal(-0.5, 1.0, nr))
    xc = np.exp(rng.normal(-0.5, 1.0, nc))
    yr = rng.uniform(0.1, 0.9, nr)
    yc = rng.uniform(0.1, 0.9, nc)
    p, b = _p_bip(xr, xc, yr, yc)
    R = 400
    cnt = np.zeros((nr, nc))
    wsum = np.zeros((nr, nc))
    for rep in range(R):
        src, dst, w = oracle.sample_bipartite_bf(xr, xc, yr, yc, seed=15, replica=rep)
        np.add.at(cnt, (src, dst), 1)
        np.add.at(wsum, (src, dst), w)
    ok = p * R > 5
    z = (cnt / R - p) / np.sqrt(p * (1 - p) / R)
    assert stats.chi2.sf((z[ok] ** 2).sum(), ok.sum()) > 1e-6
    # E[w_ij] = p/(1-b) (0 without an edge); Var = p(1+b)/(1-b)^2 - E^2
    ew = p / (1 - b)
    vw = p * (1 + b) / (1 - b) ** 2 - ew ** 2
    zw = (wsum / R - ew) / np.sqrt(vw / R)
    assert stats.chi2.sf((zw[ok] ** 2).sum(), ok.sum()) > 1e-6
    src, dst, _ = oracle.sample_bipartite_bf(xr[:20], xc[:20], exclude_self=True, seed=15, replica=0)
    assert np.all(src != dst)


def test_bipartite_edge_order_and_ids():
    rng = np.random.default_rng(180)
    nr, nc = 200, 300
    xr = np.exp(rng.normal(-2.0, 1.5, nr))
    xc = np.exp(rng.normal(-2.0, 1.5, nc))
    s = oracle.sample_bipartite(xr, xc, seed=3, replica=1, seg_work=4)
    rank_r = np.empty(nr, np.int64)
    rank_r[_order(xr)] = np.arange(nr)
    rank_c = np.empty(nc, np.int64)
    rank_c[_order(xc)] = np.arange(nc)
    key = rank_r[s.src] * nc + rank_c[s.dst]
    assert np.all(np.diff(key) > 0)  # canonical order: row rank, then column rank; no duplicates
    assert s.stats["accepts"] == s.n_edges


@pytest.mark.parametrize("seg_work", [1, 3, 32])
def test_bipartite_plan_partitions_columns(seg_work):
    rng = np.random.default_rng(190 + seg_work)
    nr, nc = 60, 400
    xr = np.exp(rng.normal(-1, 1.5, nr))
    yr = rng.uniform(0.2, 0.9, nr)
    xc = np.exp(rng.normal(-2, 1.5, nc))
    yc = rng.uniform(0.2, 0.9, nc)
    zc = xc * yc
    zcs = zc[_order(zc)]
    P = np.concatenate([[0], np.cumsum([(1 << 32) if z >= 1 else int(z * 2.0 ** 32) for z in zcs])]).astype(object)
    for i in range(nr):
        s = xr[i] * yr[i]
        c = 1.0 - yr[i] * yc.max()
        a, b = oracle.plan_row_bipartite(zcs, s, c, seg_work)
        assert a[0] == 0 and b[-1] == nc
        assert np.all(a[1:] == b[:-1])
        J = next((j for j in range(nc) if s * zcs[j] < c), nc)
        nd = -(-J // seg_work)
        assert np.all(b[:nd] - a[:nd] <= seg_work)
        if nd:
            assert b[nd - 1] == J
        if J < nc:
            md = (float(seg_work) * c / s) * 4294967296.0
            m = max(1, min(int(md), 1 << 62)) if md < 2.0 ** 62 else 1 << 62
            for k in range(nd + 1, len(a)):
                thr = P[J] + (k - nd) * m
                assert a[k] == next(j for j in range(J, nc + 1) if P[j] >= thr)
    a, b = oracle.plan_row_bipartite(zcs, 0.0, 1.0, seg_work)
    assert len(a) == 0
    a, b = oracle.plan_row_bipartite(zcs, 1.0, 1.0, 0)
    assert list(a) == [0] and list(b) == [nc]


def test_bipartite_invalid_and_empty():
    one = np.ones(3)
    with pytest.raises(ValueError):
        oracle.sample_bipartite(np.array([1.0, -1.0]), one)
    with pytest.raises(ValueError):
        oracle.sample_bipartite(one, np.array([np.nan]))
    with pytest.raises(ValueError):
        oracle.sample_bipartite(one, one, np.full(3, 0.99), np.full(3, 1.02))  # y+ y- >= 1
    with pytest.raises(ValueError):
        oracle.sample_bipartite(np.array([1e200]), np.array([1e200]))  # t overflows
    assert oracle.sample_bipartite(np.zeros(0), one).n_edges == 0
    assert oracle.sample_bipartite(one, np.zeros(0)).n_edges == 0
    assert oracle.sample_bipartite(np.zeros(5), one).n_edges == 0
    # y+ y- < 1 is all that is needed: y+ alone may exceed 1
    s = oracle.sample_bipartite(one, one, np.full(3, 1.5), np.full(3, 0.5), seed=1)
    assert np.all(s.w >= 1)
