"""Pins of the oracle's expected degree / strength and of its gradient."""
import numpy as np
import pytest

import oracle


def test_constant_x_closed_form():
    n, x = 500, 0.37
    k, _ = oracle.expected_degree(np.full(n, x))
    assert np.allclose(k, (n - 1) * x * x / (1 + x * x), rtol=1e-14, atol=0)


def test_two_block_closed_form_weighted():
    # two groups (na nodes at (xa, ya), nb at (xb, yb)); closed form by hand
    na, nb = 7, 5
    xa, ya, xb, yb = 1.3, 0.4, 0.2, 0.8
    x = np.array([xa] * na + [xb] * nb)
    y = np.array([ya] * na + [yb] * nb)

    def pe(xi, yi, xj, yj):
        a, b = xi * xj, yi * yj
        p = a * b / (1 - b + a * b)
        return p, p / (1 - b)

    paa, eaa = pe(xa, ya, xa, ya)
    pab, eab = pe(xa, ya, xb, yb)
    pbb, ebb = pe(xb, yb, xb, yb)
    k, s = oracle.expected_degree(x, y)
    assert np.allclose(k[:na], (na - 1) * paa + nb * pab, rtol=1e-14)
    assert np.allclose(k[na:], na * pab + (nb - 1) * pbb, rtol=1e-14)
    assert np.allclose(s[:na], (na - 1) * eaa + nb * eab, rtol=1e-14)
    assert np.allclose(s[na:], na * eab + (nb - 1) * ebb, rtol=1e-14)


@pytest.mark.parametrize("weighted", [False, True])
def test_class_multiplicity_equals_expansion(weighted):
    rng = np.random.default_rng(3)
    K = 30
    xc = np.exp(rng.normal(-1, 1, K))
    yc = rng.uniform(0.1, 0.9, K) if weighted else None
    m = rng.integers(1, 6, K)
    x = np.repeat(xc, m)
    y = np.repeat(yc, m) if weighted else None
    kf, sf = oracle.expected_degree(x, y)
    kc, sc = oracle.expected_degree(xc, yc, mult=m.astype(float))
    first = np.concatenate([[0], np.cumsum(m)[:-1]])
    assert np.allclose(kc, kf[first], rtol=1e-13)
    if weighted:
        assert np.allclose(sc, sf[first], rtol=1e-13)
    # L = sum_c g_c k_c over classes is the expanded L with upstream g_c / m_c on
    # each member; the gradient of a shared class parameter sums its members'.
    gk = rng.normal(size=K)
    gs = rng.normal(size=K) if weighted else None
    gxc, gyc = oracle.expected_degree_grad(xc, yc, m.astype(float), gk, gs)
    gxf, gyf = oracle.expected_degree_grad(x, y, None, np.repeat(gk / m, m),
                                           None if gs is None else np.repeat(gs / m, m))
    summed = np.add.reduceat(gxf, first)
    assert np.allclose(gxc, summed, rtol=1e-10)
    if weighted:
        assert np.allclose(gyc, np.add.reduceat(gyf, first), rtol=1e-10)


def _log_partition(x, y):
    """F = sum_{i<j} log(1 + x_i x_j) (UBCM) or log((1 - b + ab)/(1 - b)) (UECM).

    d F / d log x_i = k_i and d F / d log y_i = s_i (maximum-entropy identity)."""
    n = len(x)
    a = np.outer(x, x)
    iu = np.triu_indices(n, 1)
    if y is None:
        return np.log1p(a[iu]).sum()
    b = np.outer(y, y)
    return (np.log1p(a[iu] * b[iu] / (1 - b[iu]))).sum()


@pytest.mark.parametrize("weighted", [False, True])
def test_degree_is_gradient_of_log_partition(weighted):
    rng = np.random.default_rng(4)
    n = 40
    x = np.exp(rng.normal(-0.5, 1, n))
    y = rng.uniform(0.1, 0.9, n) if weighted else None
    k, s = oracle.expected_degree(x, y)
    h = 1e-6
    for i in range(0, n, 7):
        e = np.zeros(n)
        e[i] = h
        fd = (_log_partition(x * np.exp(e), y) - _log_partition(x * np.exp(-e), y)) / (2 * h)
        assert abs(fd - k[i]) <= 1e-7 * max(1, abs(k[i]))
        if weighted:
            fd = (_log_partition(x, y * np.exp(e)) - _log_partition(x, y * np.exp(-e))) / (2 * h)
            assert abs(fd - s[i]) <= 1e-7 * max(1, abs(s[i]))


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_central_differences(weighted):
    rng = np.random.default_rng(5)
    n = 60
    x = np.exp(rng.normal(-0.5, 1, n))
    y = rng.uniform(0.1, 0.9, n) if weighted else None
    gk = rng.normal(size=n)
    gs = rng.normal(size=n) if weighted else None

    def L(xx, yy):
        k, s = oracle.expected_degree(xx, yy)
        v = (gk * k).sum()
        if weighted:
            v += (gs * s).sum()
        return v

    gx, gy = oracle.expected_degree_grad(x, y, None, gk, gs)
    for i in range(n):
        h = 1e-6 * x[i]
        e = np.zeros(n)
        e[i] = h
        fd = (L(x + e, y) - L(x - e, y)) / (2 * h)
        assert abs(fd - gx[i]) <= 1e-6 * max(1.0, abs(gx[i]))
        if weighted:
            h = 1e-6 * y[i]
            e = np.zeros(n)
            e[i] = h
            fd = (L(x, y + e) - L(x, y - e)) / (2 * h)
            assert abs(fd - gy[i]) <= 1e-6 * max(1.0, abs(gy[i]))


def test_selected_rows_match_full():
    rng = np.random.default_rng(6)
    x = np.exp(rng.normal(-1, 1, 300))
    y = rng.uniform(0.1, 0.9, 300)
    kf, sf = oracle.expected_degree(x, y)
    rows = np.array([0, 17, 299, 150])
    k, s = oracle.expected_degree(x, y, rows=rows)
    assert np.array_equal(k, kf[rows]) and np.array_equal(s, sf[rows])
