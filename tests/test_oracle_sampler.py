"""Statistical and structural pins of the C oracle's samplers.

The exact law is the brute-force model of Sec. 2.2 / 2.5: every pair {i, j} is
an edge independently with probability p_ij, and for the weighted model the
weight given an edge is geometric with P(w) = b^(w-1) (1 - b).
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def _p_ubcm(x):
    t = np.outer(x, x)
    return t / (1.0 + t)


def _p_uecm(x, y):
    z = x * y
    t = np.outer(z, z)
    b = np.outer(y, y)
    return t / (1.0 - b + t), b


def _joint_chi2(samples_fn, n, p, R):
    """Chi-square of the full joint law of the n(n-1)/2 pair indicators."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    idx = {pr: k for k, pr in enumerate(pairs)}
    counts = np.zeros(2 ** len(pairs))
    for rep in range(R):
        src, dst = samples_fn(rep)
        code = 0
        for a, b in zip(src, dst):
            i, j = (a, b) if a < b else (b, a)
            code |= 1 << idx[(i, j)]
        counts[code] += 1
    probs = np.ones(2 ** len(pairs))
    for k, (i, j) in enumerate(pairs):
        bit = (np.arange(2 ** len(pairs)) >> k) & 1
        probs *= np.where(bit == 1, p[i, j], 1.0 - p[i, j])
    exp = probs * R
    keep = exp >= 5
    chi = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    # fold the sparse cells into one
    rest_o, rest_e = counts[~keep].sum(), exp[~keep].sum()
    dof = keep.sum() - 1
    if rest_e > 0:
        chi += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    return stats.chi2.sf(chi, dof)


@pytest.mark.parametrize("seg_work", [0, 1])
def test_ubcm_joint_law_chi2(seg_work):
    rng = np.random.default_rng(21)
    n = 5
    x = np.exp(rng.normal(-0.3, 1.0, n))
    p = _p_ubcm(x)

    def fn(rep):
        s = oracle.sample_mh(x, None, seed=77, replica=rep, seg_work=seg_work, capacity=64)
        return s.src, s.dst

    assert _joint_chi2(fn, n, p, 40_000) > 1e-6


@pytest.mark.parametrize("seg_work", [0, 1])
def test_uecm_joint_law_and_weights(seg_work):
    rng = np.random.default_rng(22)
    n = 5
    x = np.exp(rng.normal(0.5, 1.0, n))
    y = rng.uniform(0.1, 0.85, n)
    p, b = _p_uecm(x, y)
    W = {}

    def fn(rep):
        s = oracle.sample_mh(x, y, seed=78, replica=rep, seg_work=seg_work, capacity=64)
        for a, c, w in zip(s.src, s.dst, s.w):
            key = (min(a, c), max(a, c))
            W.setdefault(key, []).append(int(w))
        return s.src, s.dst

    assert _joint_chi2(fn, n, p, 40_000) > 1e-6
    # weight law given an edge: P(w) = b^(w-1)(1-b), w >= 1
    for (i, j), ws in W.items():
        ws = np.array(ws)
        bij = b[i, j]
        kmax = 8
        obs = np.array([np.sum(ws == k) for k in range(1, kmax)] + [np.sum(ws >= kmax)], dtype=float)
        pk = np.array([bij ** (k - 1) * (1 - bij) for k in range(1, kmax)] + [bij ** (kmax - 1)])
        e = pk * len(ws)
        keep = e >= 5
        chi = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum()
        assert stats.chi2.sf(chi, max(keep.sum() - 1, 1)) > 1e-6


def test_proposal_count_matches_exact_law():
    # Expected candidates per sample from the exact path law (q moves to the
    # evaluated column's probability after every candidate, Sec. 2.3).
    from oracle import enumerate as en

    rng = np.random.default_rng(23)
    n = 7
    x = np.exp(rng.normal(0.3, 1.0, n))
    perm, zs, _, _ = oracle.sorted_params(x)
    mean, var = 0.0, 0.0
    for r in range(n - 1):
        p = {j: en.ubcm_p(zs[r] * zs[j]) for j in range(r, n)}
        law = en.segment_proposals(p, p, r + 1, n, p[r])
        m1 = sum(k * w for k, w in law.items())
        m2 = sum(k * k * w for k, w in law.items())
        mean += float(m1)
        var += float(m2 - m1 * m1)
    R = 20_000
    props = [oracle.sample_mh(x, None, seed=12, replica=rep, capacity=64).stats["proposals"] for rep in range(R)]
    assert abs(np.mean(props) - mean) <= 4 * np.sqrt(var / R)


def test_ubcm_mean_degree_4sigma_n2000():
    from workloads import cfg1_small

    x = cfg1_small(seed=1)
    n = len(x)
    k_exp, _ = oracle.expected_degree(x)
    P = _p_ubcm(x)
    np.fill_diagonal(P, 0.0)
    var = (P * (1 - P)).sum(axis=1)
    R = 300
    deg = np.zeros(n)
    m_tot = []
    for rep in range(R):
        s = oracle.sample_mh(x, None, seed=5, replica=rep, seg_work=0)
        deg += np.bincount(s.src, minlength=n) + np.bincount(s.dst, minlength=n)
        m_tot.append(s.n_edges)
    z = (deg / R - k_exp) / np.sqrt(var / R)
    assert np.mean(np.abs(z) > 4) < 0.002
    assert stats.chi2.sf((z ** 2).sum(), n) > 1e-6
    M = k_exp.sum() / 2
    vm = (P * (1 - P)).sum() / 2
    assert abs(np.mean(m_tot) - M) <= 4 * np.sqrt(vm / R)


def test_uecm_mean_strength_4sigma():
    from workloads import powerlaw_degrees, uecm_recipe

    rng = np.random.default_rng(9)
    n = 1500
    k = powerlaw_degrees(rng, n, 2.3, 1, 100)
    s = np.rint(k * (1 + rng.gamma(2.0, 3.0, n))).astype(np.int64)
    x, y = uecm_recipe(k, s)
    ek, es = oracle.expected_degree(x, y)
    P, B = _p_uecm(x, y)
    np.fill_diagonal(P, 0.0)
    # Var of w_ij (0 without an edge): E[w^2] - E[w]^2, E[w] = p/(1-b), E[w^2] = p(1+b)/(1-b)^2
    varw = P * (1 + B) / (1 - B) ** 2 - (P / (1 - B)) ** 2
    R = 200
    deg = np.zeros(n)
    stren = np.zeros(n)
    for rep in range(R):
        smp = oracle.sample_mh(x, y, seed=6, replica=rep, seg_work=8)
        deg += np.bincount(smp.src, minlength=n) + np.bincount(smp.dst, minlength=n)
        stren += np.bincount(smp.src, weights=smp.w, minlength=n) + np.bincount(smp.dst, weights=smp.w, minlength=n)
    zk = (deg / R - ek) / np.sqrt((P * (1 - P)).sum(axis=1) / R)
    zs = (stren / R - es) / np.sqrt(varw.sum(axis=1) / R)
    assert np.mean(np.abs(zk) > 4) < 0.003
    assert np.mean(np.abs(zs) > 4) < 0.003
    assert stats.chi2.sf((zk ** 2).sum(), n) > 1e-6


def test_homogeneous_parameters_accept_every_proposal():
    # Identical x (the Erdos-Renyi case of Sec. 2.3): q == p at every step.
    x = np.full(300, 0.1)
    smp = oracle.sample_mh(x, None, seed=3, replica=0, seg_work=0)
    assert smp.stats["accepts"] == smp.stats["proposals"] > 0
    # edge count ~ Binomial(N(N-1)/2, p) over replicas
    p = 0.01 / 1.01
    npairs = 300 * 299 // 2
    counts = [oracle.sample_mh(x, None, seed=3, replica=r).n_edges for r in range(200)]
    assert abs(np.mean(counts) - npairs * p) <= 4 * np.sqrt(npairs * p * (1 - p) / 200)


def test_constant_y_bound_is_tight():
    # Homogeneous beta (Sec. 4): the bound equals the true probability, so every
    # proposal is accepted with ratio p/q where q is the previous column's p.
    rng = np.random.default_rng(4)
    x = np.exp(rng.normal(0, 1, 40))
    y = np.full(40, 0.6)
    perm, zs, ys, c = oracle.sorted_params(x, y)
    assert np.all(c[:-1] == 1.0 - 0.6 * 0.6)


@pytest.mark.parametrize("seg_work", [0, 1, 4, 64])
def test_bf_and_mh_agree_in_distribution(seg_work):
    rng = np.random.default_rng(31)
    n = 60
    x = np.exp(rng.normal(-1.0, 1.2, n))
    P = _p_ubcm(x)
    np.fill_diagonal(P, 0)
    R = 300
    cnt_mh = np.zeros((n, n))
    for rep in range(R):
        s = oracle.sample_mh(x, None, seed=9, replica=rep, seg_work=seg_work)
        cnt_mh[s.src, s.dst] += 1
    cnt_mh = cnt_mh + cnt_mh.T
    iu = np.triu_indices(n, 1)
    z = (cnt_mh[iu] / R - P[iu]) / np.sqrt(np.maximum(P[iu] * (1 - P[iu]), 1e-12) / R)
    ok = P[iu] * R > 5
    assert stats.chi2.sf((z[ok] ** 2).sum(), ok.sum()) > 1e-6


def test_bf_pair_marginals():
    rng = np.random.default_rng(32)
    n = 40
    x = np.exp(rng.normal(-1.0, 1.2, n))
    P = _p_ubcm(x)
    R = 400
    cnt = np.zeros((n, n))
    for rep in range(R):
        src, dst, _, _ = oracle.sample_bf(x, None, seed=10, replica=rep)
        assert np.all(src < dst)
        cnt[src, dst] += 1
    iu = np.triu_indices(n, 1)
    ok = P[iu] * R > 5
    z = (cnt[iu] / R - P[iu]) / np.sqrt(P[iu] * (1 - P[iu]) / R)
    assert stats.chi2.sf((z[ok] ** 2).sum(), ok.sum()) > 1e-6


def test_bf_row_ranges_concatenate():
    rng = np.random.default_rng(33)
    x = np.exp(rng.normal(-2, 1, 100))
    full = oracle.sample_bf(x, None, seed=1, replica=2)
    parts = [oracle.sample_bf(x, None, seed=1, replica=2, row_begin=a, row_end=a + 25) for a in range(0, 100, 25)]
    assert np.array_equal(full[0], np.concatenate([p[0] for p in parts]))
    assert np.array_equal(full[1], np.concatenate([p[1] for p in parts]))


def test_order_matches_lexsort():
    rng = np.random.default_rng(40)
    z = np.round(rng.exponential(1.0, 5000), 2)  # many ties
    perm = oracle.order(z)
    ref = np.lexsort((np.arange(len(z)), -z))
    assert np.array_equal(perm, ref)


def test_bound_brute_force():
    rng = np.random.default_rng(41)
    ys = rng.uniform(0, 1, 200)
    c = oracle.bound(ys)
    for r in range(len(ys)):
        tail = np.sort(ys[r:])[::-1]
        Y = tail[0] * tail[1] if len(tail) >= 2 else 0.0
        assert c[r] == 1.0 - Y


@pytest.mark.parametrize("seg_work", [1, 3, 32])
def test_plan_partitions_rows(seg_work):
    rng = np.random.default_rng(50 + seg_work)
    n = 400
    x = np.exp(rng.normal(-2, 1.5, n))
    y = rng.uniform(0.2, 0.9, n)
    perm, zs, ys, c = oracle.sorted_params(x, y)
    counts = oracle.plan_counts(zs, c, seg_work)
    P = np.concatenate([[0], np.cumsum([(1 << 32) if z >= 1 else int(z * 2.0 ** 32) for z in zs])]).astype(object)
    for r in range(n - 1):
        a, b = oracle.plan_row(zs, c, seg_work, r)
        assert len(a) == counts[r] >= 1
        assert a[0] == r + 1 and b[-1] == n
        assert np.all(a[1:] == b[:-1])
        # linear-scan recomputation of the dense end J and of the mass cuts
        J = next((j for j in range(r + 1, n) if zs[r] * zs[j] < c[r]), n)
        nd = -(-(J - r - 1) // seg_work)
        assert np.all(b[:nd] - a[:nd] <= seg_work)
        if nd:
            assert b[nd - 1] == J
        if J < n:
            md = (float(seg_work) * c[r] / zs[r]) * 4294967296.0
            m = max(1, min(int(md), 1 << 62)) if md < 2.0 ** 62 else 1 << 62
            for k in range(nd + 1, len(a)):
                thr = P[J] + (k - nd) * m
                jj = next(j for j in range(J, n + 1) if P[j] >= thr)
                assert a[k] == jj
    assert counts[n - 1] == 0


def test_unsegmented_plan_is_one_segment():
    rng = np.random.default_rng(60)
    x = np.exp(rng.normal(0, 2, 100))
    perm, zs, _, _ = oracle.sorted_params(x)
    counts = oracle.plan_counts(zs, None, 0)
    assert np.all(counts[:-1] == 1) and counts[-1] == 0


def test_invalid_parameters_rejected():
    with pytest.raises(ValueError):
        oracle.sample_mh(np.array([1.0, -1.0, 0.5]))
    with pytest.raises(ValueError):
        oracle.sample_mh(np.array([1.0, np.nan]))
    with pytest.raises(ValueError):
        oracle.sample_mh(np.array([1.0, 2.0]), np.array([1.1, 0.95]))  # y1*y2 >= 1
    with pytest.raises(ValueError):
        oracle.sample_mh(np.array([1e200, 1e200]))  # t overflows


def test_zero_and_tiny_inputs():
    assert oracle.sample_mh(np.zeros(10)).n_edges == 0
    assert oracle.sample_mh(np.array([3.0])).n_edges == 0
    assert oracle.sample_mh(np.zeros(0)).n_edges == 0


def test_capacity_retry_identical():
    x = np.exp(np.random.default_rng(5).normal(-1, 1, 200))
    full = oracle.sample_mh(x, None, seed=2, replica=1, seg_work=4)
    small = oracle.sample_mh(x, None, seed=2, replica=1, seg_work=4, capacity=3)
    assert np.array_equal(full.src, small.src) and np.array_equal(full.dst, small.dst)


# ------------------------------------------------------------------ skip law (Sec. 2.3)
def _u53_draws(seed: int, n: int) -> np.ndarray:
    # uniforms on the sampler's grid {k 2^-53 : k = 1 .. 2^53}
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 1 << 53, size=n, dtype=np.int64).astype(np.float64) + 1.0) * 2.0 ** -53


@pytest.mark.parametrize("tq,c", [(0.05, 1.0), (1.0, 1.0), (20.0, 1.0), (0.3, 0.55), (4.0, 0.2)])
def test_skip_law_chi2(tq, c):
    # floor(d) is geometric on {0, 1, ...} with P(L = l) = (1 - q)^l q and
    # q = t_q / (c + t_q): the proposal probability of Sec. 2.3 (unweighted,
    # c = 1) or the weighted bound of Sec. 2.5 (c = 1 - Y)
    R = 200_000
    L = np.floor(oracle.skip_reals(_u53_draws(int(tq * 1000 + c * 10), R), tq, c))
    assert np.all(L >= 0)
    q = tq / (c + tq)
    lmax = int(np.ceil(np.log(5.0 / R) / np.log1p(-q))) if q < 1 else 1
    lmax = max(1, min(lmax, 400))
    obs = np.array([np.sum(L == l) for l in range(lmax)] + [np.sum(L >= lmax)], dtype=float)
    pl = np.array([(1 - q) ** l * q for l in range(lmax)] + [(1 - q) ** lmax])
    e = pl * R
    keep = e >= 5
    chi = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum() + (obs[~keep].sum() - e[~keep].sum()) ** 2 / max(
        e[~keep].sum(), 1e-300) * (e[~keep].sum() > 0)
    assert stats.chi2.sf(chi, max(int(keep.sum()), 1)) > 1e-6


@pytest.mark.parametrize("q,c", [(1e-9, 1.0), (1e-9, 0.3), (1e-18, 1.0), (1e-150, 1.0)])
def test_skip_mean_at_tiny_q(q, c):
    # mean of the geometric skip is (1 - q)/q, its variance (1 - q)/q^2: within
    # 4 sigma over R draws, at proposal probabilities where 1 - q rounds to 1 in
    # binary64 (a skip computed from log(1 - q) would never end)
    R = 400_000
    tq = c * q / (1.0 - q)
    L = np.floor(oracle.skip_reals(_u53_draws(7, R), tq, c))
    mean = (1.0 - q) / q
    sigma = np.sqrt((1.0 - q) / q ** 2 / R)
    assert np.all(np.isfinite(L))
    assert abs(L.mean() - mean) <= 4 * sigma


@pytest.mark.parametrize("c", [1.0, 0.25])
def test_skip_at_q_near_one(c):
    # q = 1 - 1e-9: the next column is proposed unless U1 <= 1 - q, i.e. with
    # probability q; L = 0 exactly when -log U1 < log1p(t_q / c).  Every draw
    # of 400,000 gives L = 0 except with probability 4e-4, and the mean
    # (1 - q)/q = 1e-9 is within 4 sigma (sigma = 5e-8) only then.
    q = 1.0 - 1e-9
    tq = c * q / (1.0 - q)
    R = 400_000
    L = np.floor(oracle.skip_reals(_u53_draws(8, R), tq, c))
    assert abs(L.mean() - (1 - q) / q) <= 4 * np.sqrt((1 - q) / q ** 2 / R)
    # the boundary itself: U1 just above and at 1/(1 + t_q / c)
    thr = 1.0 / (1.0 + tq / c)
    k = np.floor(thr * 2.0 ** 53)
    assert np.floor(oracle.skip_reals([(k + 2) * 2.0 ** -53], tq, c))[0] == 0
    assert np.floor(oracle.skip_reals([(k - 2) * 2.0 ** -53], tq, c))[0] >= 1


def test_skip_endpoints_and_monotone():
    # U1 = 1 gives d = 0 (the next column); d falls as U1 grows
    d = oracle.skip_reals([1.0], 0.7, 1.0)
    assert d[0] == 0.0
    u = np.sort(_u53_draws(9, 2000))
    d = oracle.skip_reals(u, 0.7, 0.8)
    assert np.all(np.diff(d) <= 0)
    assert np.allclose(d, -np.log(u) / np.log1p(0.7 / 0.8), rtol=1e-15)


# ------------------------------------------------------------------ weighted brute force (Secs. 2.2, 2.5)
def test_weighted_bf_joint_law_and_weights():
    # one node set, weighted: every pair an edge independently with
    # p = t / (1 - b + t), and given the edge w ~ b^(w-1)(1 - b), w >= 1
    rng = np.random.default_rng(24)
    n = 5
    x = np.exp(rng.normal(0.5, 1.0, n))
    y = rng.uniform(0.3, 0.85, n)
    p, b = _p_uecm(x, y)
    W = {}

    def fn(rep):
        src, dst, w, _ = oracle.sample_bf(x, y, seed=81, replica=rep)
        for a, c, ww in zip(src, dst, w):
            assert a < c
            W.setdefault((int(a), int(c)), []).append(int(ww))
        return src, dst

    assert _joint_chi2(fn, n, p, 40_000) > 1e-6
    assert len(W) == n * (n - 1) // 2
    for (i, j), ws in W.items():
        ws = np.array(ws)
        bij = b[i, j]
        kmax = 10
        obs = np.array([np.sum(ws == k) for k in range(1, kmax)] + [np.sum(ws >= kmax)], dtype=float)
        pk = np.array([bij ** (k - 1) * (1 - bij) for k in range(1, kmax)] + [bij ** (kmax - 1)])
        e = pk * len(ws)
        keep = e >= 5
        chi = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum()
        assert stats.chi2.sf(chi, max(keep.sum() - 1, 1)) > 1e-6, (i, j)
        # the mean weight 1 / (1 - b): within 4 sigma (variance b / (1 - b)^2)
        assert abs(ws.mean() - 1 / (1 - bij)) <= 4 * np.sqrt(bij / (1 - bij) ** 2 / len(ws))


def test_weighted_bf_mean_strength_4sigma():
    # the brute force's strengths over replicas against s_i = sum_j p_ij / (1 - b_ij)
    rng = np.random.default_rng(25)
    n = 400
    x = np.exp(rng.normal(-1.5, 1.0, n))
    y = rng.uniform(0.2, 0.9, n)
    ek, es = oracle.expected_degree(x, y)
    P, B = _p_uecm(x, y)
    np.fill_diagonal(P, 0.0)
    varw = P * (1 + B) / (1 - B) ** 2 - (P / (1 - B)) ** 2
    R = 200
    deg = np.zeros(n)
    stren = np.zeros(n)
    for rep in range(R):
        src, dst, w, _ = oracle.sample_bf(x, y, seed=12, replica=rep)
        deg += np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
        stren += np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    zk = (deg / R - ek) / np.sqrt((P * (1 - P)).sum(axis=1) / R)
    zs = (stren / R - es) / np.sqrt(varw.sum(axis=1) / R)
    assert stats.chi2.sf((zk ** 2).sum(), n) > 1e-6
    assert stats.chi2.sf((zs ** 2).sum(), n) > 1e-6
