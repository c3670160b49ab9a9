"""Pins of the oracle's random-number layer: Philox4x32-10 and the 53-bit uniform."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(tok, 16) for tok in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox(ctr, key)) == expect


def test_philox_counter_sensitivity():
    # Each counter word and each key word changes every output word (avalanche).
    base = oracle.philox([1, 2, 3, 4], [5, 6])
    for pos in range(4):
        c = [1, 2, 3, 4]
        c[pos] ^= 1
        out = oracle.philox(c, [5, 6])
        assert np.all(out != base)
    for pos in range(2):
        k = [5, 6]
        k[pos] ^= 1
        assert np.all(oracle.philox([1, 2, 3, 4], k) != base)


def test_u53_range_endpoints():
    # (((a << 21) | (b >> 11)) + 1) * 2^-53 lies in (0, 1]
    assert oracle.u53(0, 0) == 2.0 ** -53
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    assert oracle.u53(0x80000000, 0) == 0.5 + 2.0 ** -53
    # low 11 bits of b are discarded
    assert oracle.u53(7, 0x7FF) == oracle.u53(7, 0)
    assert oracle.u53(7, 0x800) == oracle.u53(7, 0) + 2.0 ** -53


def test_u53_uniform_ks():
    # Kolmogorov-Smirnov on 20k uniforms drawn through consecutive counters.
    u = []
    for s in range(10_000):
        w = oracle.philox([s, 17, 0, 0], [123, 456])
        u.append(oracle.u53(int(w[0]), int(w[1])))
        u.append(oracle.u53(int(w[2]), int(w[3])))
    res = stats.kstest(np.array(u), "uniform")
    assert res.pvalue > 1e-4
