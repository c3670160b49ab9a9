"""Pins of the oracle's Chung-Lu sampler and of the network statistics used to
show the Chung-Lu model's bias (Sec. 2.1: rich-club density, Fig. 1A;
triangle counts, Fig. 1B; Sec. 2.3: the Miller-Hagberg chain for the Chung-Lu
model, p_ij = min(w_i w_j, 1)).

The exact law of the Chung-Lu model read as edge probabilities is: every
pair {i, j} is an edge independently with probability min(w_i w_j, 1).
"""
from itertools import combinations

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enumerate as en
from test_oracle_sampler import _joint_chi2


def _sorted_w(seed, n, mu=0.0, sd=1.0):
    rng = np.random.default_rng(seed)
    w = np.exp(rng.normal(mu, sd, n))
    perm, zs, _, _ = oracle.sorted_params(w)
    return w, zs


# ------------------------------------------------------------------ the chain, exactly
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chung_lu_rows_exact(seed):
    # products on both sides of 1: runs of columns with q = 1, then q < 1
    _, zs = _sorted_w(seed, 7, mu=-0.3)
    assert (zs[0] * zs[1] > 1.0) and (zs[-2] * zs[-1] < 1.0)
    for r in range(len(zs) - 1):
        law, target = en.row_law(list(zs), r, [(r + 1, len(zs))], chung_lu=True)
        assert law == target


@pytest.mark.parametrize("seed", [3, 4])
def test_chung_lu_segmented_rows_exact(seed):
    _, zs = _sorted_w(seed, 7, mu=0.2)
    n = len(zs)
    for r in range(n - 2):
        for cut in range(r + 2, n):
            law, target = en.row_law(list(zs), r, [(r + 1, cut), (cut, n)], chung_lu=True)
            assert law == target


def test_chung_lu_plan_segments_exact():
    # rows cut by the oracle's own plan rule (c = 1) stay exact
    _, zs = _sorted_w(11, 7, mu=0.4)
    n = len(zs)
    seen = False
    for r in range(n - 1):
        a, b = oracle.plan_row(zs, None, 1, r)
        segs = [(int(u), int(v)) for u, v in zip(a, b)]
        seen |= len(segs) > 1
        law, target = en.row_law(list(zs), r, segs, chung_lu=True)
        assert law == target
    assert seen


def test_chung_lu_chain_with_a_smaller_proposal_is_biased():
    # negative control: proposing with the UBCM probability t / (1 + t), which
    # lies below min(t, 1), breaks the bound and the law
    _, zs = _sorted_w(5, 6)
    n = len(zs)
    s = zs[0]
    p = {j: en.chung_lu_p(s * zs[j]) for j in range(n)}
    q = {j: en.ubcm_p(s * zs[j]) for j in range(n)}
    law = en.segment_law(p, q, 1, n, q[0])
    assert law != en.bernoulli_law(p, list(range(1, n)))


# ------------------------------------------------------------------ the C sampler
@pytest.mark.parametrize("seg_work", [0, 1])
def test_chung_lu_joint_law_chi2(seg_work):
    rng = np.random.default_rng(31)
    n = 5
    w = np.exp(rng.normal(-0.2, 0.9, n))
    t = np.outer(w, w)
    p = np.minimum(t, 1.0)
    assert (p == 1.0).sum() > n and (p < 0.5).any()  # some pairs certain, some not

    def fn(rep):
        s = oracle.sample_chung_lu(w, seed=91, replica=rep, seg_work=seg_work, capacity=64)
        return s.src, s.dst

    assert _joint_chi2(fn, n, p, 40_000) > 1e-6


def test_chung_lu_mean_degree_4sigma():
    # E[deg_i] = sum_j min(w_i w_j, 1), Var = sum_j p (1 - p): 4 sigma over replicas
    rng = np.random.default_rng(32)
    n = 1500
    k = workloads_powerlaw(rng, n)
    w = k / np.sqrt(k.sum())
    t = np.outer(w, w)
    np.fill_diagonal(t, 0.0)
    p = np.minimum(t, 1.0)
    E = p.sum(1)
    V = (p * (1 - p)).sum(1)
    R = 400
    deg = np.zeros(n)
    for rep in range(R):
        s = oracle.sample_chung_lu(w, seed=5, replica=rep, seg_work=4)
        deg += np.bincount(s.src, minlength=n) + np.bincount(s.dst, minlength=n)
    z = (deg / R - E) / np.sqrt(V / R + 1e-300)
    assert np.abs(z[V > 0]).max() < 5.0
    assert np.all(deg[V == 0] == R * E[V == 0])  # certain pairs only


def workloads_powerlaw(rng, n):
    import workloads

    return workloads.powerlaw_degrees(rng, n, 2.1, 2, 300).astype(np.float64) * 3.0


def test_homogeneous_chung_lu_is_erdos_renyi():
    # constant w < 1: q == p everywhere, every proposal accepted (except
    # U2 = 1, probability 2^-53) and the edge count is Binomial(N(N-1)/2, w^2)
    n, w0 = 400, 0.11
    w = np.full(n, w0)
    counts = []
    for rep in range(200):
        s = oracle.sample_chung_lu(w, seed=3, replica=rep)
        assert s.stats["proposals"] == s.stats["accepts"]
        counts.append(s.n_edges)
    N2 = n * (n - 1) // 2
    p = w0 * w0
    mean, sd = N2 * p, np.sqrt(N2 * p * (1 - p))
    assert abs(np.mean(counts) - mean) < 4 * sd / np.sqrt(len(counts))


def test_products_above_one_give_the_complete_graph():
    w = np.linspace(1.0, 3.0, 60)
    for seg_work in (0, 1, 7):
        s = oracle.sample_chung_lu(w, seed=4, replica=1, seg_work=seg_work)
        assert s.n_edges == 60 * 59 // 2
        assert len(s.tie_rows) == 0  # a skip of 0 at q = 1 is no rounding decision


def test_chung_lu_and_ubcm_differ_where_products_are_large():
    # the same parameters under the two models: equal when every product is
    # tiny (min(t, 1) ~ t/(1+t)), Chung-Lu denser among the large ones
    w = np.exp(np.random.default_rng(7).normal(-0.5, 1.2, 800))
    cl = np.mean([oracle.sample_chung_lu(w, seed=1, replica=r).n_edges for r in range(20)])
    ub = np.mean([oracle.sample_mh(w, None, seed=1, replica=r).n_edges for r in range(20)])
    t = np.outer(w, w)
    iu = np.triu_indices(800, 1)
    assert abs(cl - np.minimum(t, 1.0)[iu].sum()) < 4 * np.sqrt(np.minimum(t, 1.0)[iu].sum() / 20)
    assert abs(ub - (t / (1 + t))[iu].sum()) < 4 * np.sqrt((t / (1 + t))[iu].sum() / 20)
    assert cl > ub


def test_invalid_chung_lu_parameters():
    for bad in ([np.nan, 1.0], [-1.0, 1.0], [np.inf, 0.5], [1e200, 1e200]):
        with pytest.raises(ValueError):
            oracle.sample_chung_lu(np.array(bad))


# ------------------------------------------------------------------ statistics
def _triangles_brute(src, dst, n):
    A = np.zeros((n, n), dtype=bool)
    A[src, dst] = True
    A[dst, src] = True
    return sum(1 for a, b, c in combinations(range(n), 3) if A[a, b] and A[a, c] and A[b, c])


def test_triangles_brute_force():
    rng = np.random.default_rng(9)
    for n, dens in ((12, 0.5), (25, 0.3), (40, 0.15), (30, 0.9)):
        iu = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
        keep = rng.random(len(iu)) < dens
        e = iu[keep]
        flip = rng.random(len(e)) < 0.5  # either orientation
        src = np.where(flip, e[:, 1], e[:, 0])
        dst = np.where(flip, e[:, 0], e[:, 1])
        o = rng.permutation(len(e))
        assert oracle.count_triangles(src[o], dst[o], n) == _triangles_brute(src, dst, n)


def test_triangles_closed_forms():
    for n in (3, 4, 10, 31):
        iu = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
        assert oracle.count_triangles(iu[:, 0], iu[:, 1], n) == n * (n - 1) * (n - 2) // 6
    for n in (4, 9, 50):  # a cycle of 4 or more nodes has none
        a = np.arange(n)
        assert oracle.count_triangles(a, (a + 1) % n, n) == 0
    # a wheel of n spokes: n triangles
    n = 12
    rim = np.arange(1, n + 1)
    src = np.concatenate([np.zeros(n, int), rim])
    dst = np.concatenate([rim, np.roll(rim, 1)])
    assert oracle.count_triangles(src, dst, n + 1) == n
    assert oracle.count_triangles(np.zeros(0, int), np.zeros(0, int), 5) == 0


def test_rank_counts_give_rich_club_edges():
    rng = np.random.default_rng(10)
    n = 60
    w = np.exp(rng.normal(-0.5, 1.0, n))
    s = oracle.sample_chung_lu(w, seed=2)
    perm = oracle.order(w)
    cnt = oracle.rank_counts(s.src, s.dst, perm)
    edges = set(zip(s.src.tolist(), s.dst.tolist()))
    for K in (1, 2, 5, 17, 60):
        top = set(perm[:K].tolist())
        brute = sum(1 for a, b in edges if a in top and b in top)
        assert cnt[:K].sum() == brute
    assert cnt.sum() == s.n_edges
