"""Exact pins of the sequential sampler (the algorithm itself, not its code).

The path tree of one row is enumerated with rational arithmetic
(oracle.enumerate) and its law of accepted columns must equal the product of
Bernoulli(p_rj) -- the brute-force model of Sec. 2.2 -- for both models, for
segmented rows, and for the bound of Sec. 2.5 read as "two largest y among the
unprocessed nodes, focal node included".  The readings not taken must fail.
"""
import numpy as np
import pytest

import oracle
from oracle import enumerate as en


def _sorted_params(seed, n, weighted):
    rng = np.random.default_rng(seed)
    x = np.exp(rng.normal(0.0, 1.0, n))
    y = rng.uniform(0.05, 0.9, n) if weighted else None
    perm, zs, ys, c = oracle.sorted_params(x, y)
    return zs, ys, c


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ubcm_rows_exact(seed):
    zs, _, _ = _sorted_params(seed, 7, False)
    for r in range(len(zs) - 1):
        law, target = en.row_law(list(zs), r, [(r + 1, len(zs))])
        assert law == target


@pytest.mark.parametrize("seed", [3, 4])
def test_ubcm_segmented_rows_exact(seed):
    zs, _, _ = _sorted_params(seed, 7, False)
    n = len(zs)
    for r in range(n - 2):
        for cut in range(r + 2, n):
            law, target = en.row_law(list(zs), r, [(r + 1, cut), (cut, n)])
            assert law == target


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_uecm_rows_exact_with_focal_bound(seed):
    zs, ys, c = _sorted_params(seed, 7, True)
    n = len(zs)
    for r in range(n - 1):
        Y = en.top2_product(ys[r:])
        assert 1.0 - Y == c[r]  # the oracle's bound is this reading
        law, target = en.row_law(list(zs), r, [(r + 1, n)], ys=list(ys), Y=Y)
        assert law == target


def test_uecm_plan_segments_exact():
    # Rows cut by the oracle's own segment rule stay exact.
    zs, ys, c = _sorted_params(11, 7, True)
    zs = zs * 3.0  # larger products: several dense columns per row
    n = len(zs)
    c = oracle.bound(ys)
    seen_split = False
    for r in range(n - 1):
        a, b = oracle.plan_row(zs, c, 1, r)
        segs = [(int(u), int(v)) for u, v in zip(a, b)]
        seen_split |= len(segs) > 1
        law, target = en.row_law(list(zs), r, segs, ys=list(ys), Y=1.0 - c[r])
        assert law == target
    assert seen_split


def test_literal_alg1_loop_order_is_biased():
    # Negative control: proposing column i+1 before any geometric draw.
    zs, _, _ = _sorted_params(0, 6, False)
    law, target = en.row_law(list(zs), 0, [(1, len(zs))], force_first=True)
    assert law != target


def test_bound_without_focal_node_is_biased():
    # Negative control: beta_min over ranks r+1.. only.  Make y_r the largest.
    zs, ys, _ = _sorted_params(8, 6, True)
    ys = np.array(ys)
    ys[0] = 0.95
    ys[1:] = np.minimum(ys[1:], 0.5)
    Y_wrong = en.top2_product(ys[1:])
    law, target = en.row_law(list(zs), 0, [(1, len(zs))], ys=list(ys), Y=Y_wrong)
    assert law != target


def test_single_min_reading_valid_when_y_below_one():
    # "minimum beta among remaining nodes" (Y = largest y) is a looser bound when y <= 1.
    zs, ys, _ = _sorted_params(9, 6, True)
    n = len(zs)
    for r in range(n - 1):
        Y = max(ys[r:])
        law, target = en.row_law(list(zs), r, [(r + 1, n)], ys=list(ys), Y=Y)
        assert law == target


def test_homogeneous_case_is_geometric_skipping():
    # Identical parameters (Sec. 2.3): every proposal has q == p, acceptance ratio 1.
    zs = [0.7] * 6
    law, target = en.row_law(zs, 0, [(1, 6)])
    assert law == target
    # the skip law alone produces the edges: P(no edge in the row) = (1-p)^5
    p = en.ubcm_p(0.7 * 0.7)
    assert law[frozenset()] == (1 - p) ** 5
