"""The sweep's logarithm (log_fast / log1p_fast in the kernel header): its
constants and series, read from the source, evaluated step by step in binary64
on the CPU and compared with the library log / log1p.  The kernel uses FMAs
where this model rounds twice, so the model's error bounds the kernel's from
above (up to the FMA's extra accuracy); parity of the sampled edges with the
oracle checks the kernel itself."""
import math
import os
import random
import re
from fractions import Fraction

import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2509_13230_amd", "csrc", "mh_common.hpp")


def _source():
    s = open(HDR).read()
    body = s[s.index("double log_reduced("):s.index("double log_fast(")]
    hi = float.fromhex(re.search(r"kLn2Hi = (0x[0-9a-fp.+-]+);", body).group(1))
    lo = float.fromhex(re.search(r"kLn2Lo = (0x[0-9a-fp.+-]+);", body).group(1))
    dens = [int(d) for d in re.findall(r"1\.0 / (\d+)\.0", body)]
    return hi, lo, dens


def _ln2():
    return sum(Fraction(1, k * 2 ** k) for k in range(1, 300))


def test_ln2_split():
    hi, lo, _ = _source()
    assert abs(Fraction(hi) + Fraction(lo) - _ln2()) < Fraction(1, 2 ** 100)
    # k * hi exact for every binary64 exponent: hi has at least 11 trailing zero bits
    m = Fraction(hi) * 2 ** 53
    assert m.denominator == 1 and int(m) % (1 << 11) == 0


def test_series_terms():
    # Horner from the highest term: 1/21, 1/19, ..., 1/3 (the odd terms after s)
    _, _, dens = _source()
    assert dens == list(range(21, 2, -2))
    # truncation after s^21 on |s| <= (sqrt2 - 1)/(sqrt2 + 1): below 2^-55 relative
    smax = (math.sqrt(2) - 1) / (math.sqrt(2) + 1)
    assert smax ** 22 / 23 < 2.0 ** -55


def _model():
    hi, lo, dens = _source()

    def reduced(m, k):
        f = m - 1.0
        s = f / (2.0 + f)
        z = s * s
        p = 1.0 / dens[0]
        for d in dens[1:]:
            p = p * z + 1.0 / d
        s2 = s + s
        return k * hi + (k * lo + (s2 * (z * p) + s2))

    def log_fast(x):
        m, k = math.frexp(x)
        if m < 0.70710678118654752440:
            m, k = m + m, k - 1
        return reduced(m, k)

    def log1p_fast(t):
        if abs(t) < 2.0 ** -27:
            return (-0.5 * t) * t + t  # the kernel's single fma rounds once; this model twice
        u = 1.0 + t
        c = t - (u - 1.0)
        return c * (1.0 / u) + log_fast(u)

    return log_fast, log1p_fast


def _ulps(a, ref):
    return abs(a - ref) / math.ulp(ref) if ref != 0.0 else abs(a)


@pytest.mark.parametrize("seed", [1, 2])
def test_model_within_a_few_ulp(seed):
    log_fast, log1p_fast = _model()
    rng = random.Random(seed)
    worst = worst1 = 0.0
    for _ in range(60_000):
        u = (rng.getrandbits(53) + 1) * 2.0 ** -53  # the sampler's uniforms
        worst = max(worst, _ulps(log_fast(u), math.log(u)))
        t = 10.0 ** rng.uniform(-14, 4)  # t_q over the range of the workloads
        worst1 = max(worst1, _ulps(log1p_fast(t), math.log1p(t)))
        t = -(10.0 ** rng.uniform(-20, -0.5))  # -t_q of the Chung-Lu skip
        worst1 = max(worst1, _ulps(log1p_fast(t), math.log1p(t)))
    for u in (2.0 ** -53, 0.5, 0.70710678118654752440, 1.0 - 2.0 ** -53):
        worst = max(worst, _ulps(log_fast(u), math.log(u)))
    assert log_fast(1.0) == 0.0
    for t in (2.0 ** -60, 1e-9, 0.41421356, 1.0, 3.0, 1e6, 2.0 ** -27, -(2.0 ** -27), -1.79e-16, -0.5):
        worst1 = max(worst1, _ulps(log1p_fast(t), math.log1p(t)))
    assert worst <= 3.0 and worst1 <= 3.0, (worst, worst1)
