"""Exact enumeration of the sequential sampler's path tree (TEST INFRASTRUCTURE).

For one source row the sampler is a Markov chain over columns: from column
``pos`` with proposal probability ``q`` it skips L ~ Geometric(q), L >= 0,
columns (Sec. 2.3: the chance that the next L candidates carry no edge is
(1-q)^L q), evaluates the candidate, accepts it with probability p/q and
moves q to the probability at that column (Sec. 2.3; Alg. 1).  Enumerating
every path with rational arithmetic gives the exact law of the row's
accepted set, which must equal the product of independent Bernoulli(p_rj)
(the brute-force model of Sec. 2.2).  Variants reproduce readings of the
paper that are *not* taken (the literal loop order of Alg. 1 and a bound that
leaves out the focal node), as negative controls.

Pure Python with fractions.Fraction: for tiny N only (row length <= ~10).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product


def F(v: float) -> Fraction:
    return Fraction(v)


def ubcm_p(t: float) -> Fraction:
    """p = t / (1 + t) for t = x_i x_j (Sec. 2.2), exactly for the float t."""
    t = F(t)
    return t / (1 + t)


def chung_lu_p(t: float) -> Fraction:
    """p = min(w_i w_j, 1): the Chung-Lu model read as edge probabilities
    (Sec. 2.1), exactly for the float t = w_i w_j."""
    return min(F(t), Fraction(1))


def uecm_p(t: float, b: float) -> Fraction:
    """p = t / (1 - b + t), t = x_i y_i x_j y_j, b = y_i y_j (Sec. 2.5)."""
    t, b = F(t), F(b)
    return t / (1 - b + t)


def uecm_bound(t: float, Y: float) -> Fraction:
    """p^ = t / (1 - Y + t), Y = exp(-beta_min) (Sec. 2.5)."""
    t, Y = F(t), F(Y)
    return t / (1 - Y + t)


def segment_law(p: dict[int, Fraction], qcol: dict[int, Fraction], a: int, b: int,
                q_start: Fraction, force_first: bool = False) -> dict[frozenset, Fraction]:
    """Law of the accepted set of columns in [a, b) for one chain segment.

    p[j]: target probability at column j; qcol[j]: proposal probability the
    chain moves to after evaluating j; q_start: proposal probability at a-1.
    force_first: evaluate column a before any geometric draw (the literal
    reading of Alg. 1's loop), a negative control.
    """
    out: dict[frozenset, Fraction] = {}

    def walk(pos: int, q: Fraction, acc: frozenset, w: Fraction):
        if w == 0:
            return
        room = b - 1 - pos  # columns left in the segment after pos
        if q == 0 or room <= 0:
            out[acc] = out.get(acc, Fraction(0)) + w
            return
        # exit: all remaining columns skipped
        stay = (1 - q) ** room
        if stay:
            out[acc] = out.get(acc, Fraction(0)) + w * stay
        for L in range(room):
            j = pos + 1 + L
            pj = w * (1 - q) ** L * q
            evaluate(j, q, acc, pj)

    def evaluate(j: int, q: Fraction, acc: frozenset, w: Fraction):
        ratio = p[j] / q
        if ratio > 1:
            ratio = Fraction(1)  # a violated bound: the sampler can only accept surely
        walk(j, qcol[j], acc | {j}, w * ratio)
        walk(j, qcol[j], acc, w * (1 - ratio))

    if a >= b:
        return {frozenset(): Fraction(1)}
    if force_first:
        evaluate(a, q_start, frozenset(), Fraction(1))
    else:
        walk(a - 1, q_start, frozenset(), Fraction(1))
    return out


def segment_proposals(p: dict[int, Fraction], qcol: dict[int, Fraction], a: int, b: int,
                      q_start: Fraction) -> dict[int, Fraction]:
    """Law of the number of candidates the chain evaluates in [a, b).

    Distinguishes chains with the same edge law but different proposal rules
    (the paper moves q to the evaluated column's probability whether or not
    the candidate was accepted)."""
    out: dict[int, Fraction] = {}

    def walk(pos: int, q: Fraction, cnt: int, w: Fraction):
        if w == 0:
            return
        room = b - 1 - pos
        if q == 0 or room <= 0:
            out[cnt] = out.get(cnt, Fraction(0)) + w
            return
        stay = (1 - q) ** room
        if stay:
            out[cnt] = out.get(cnt, Fraction(0)) + w * stay
        for L in range(room):
            j = pos + 1 + L
            walk(j, qcol[j], cnt + 1, w * (1 - q) ** L * q)

    if a < b:
        walk(a - 1, q_start, 0, Fraction(1))
    else:
        out[0] = Fraction(1)
    return out


def combine(d1: dict, d2: dict) -> dict:
    """Law of the union of two independent accepted sets on disjoint columns."""
    out: dict[frozenset, Fraction] = {}
    for s1, w1 in d1.items():
        for s2, w2 in d2.items():
            k = s1 | s2
            out[k] = out.get(k, Fraction(0)) + w1 * w2
    return out


def bernoulli_law(p: dict[int, Fraction], cols: list[int]) -> dict[frozenset, Fraction]:
    """Product of independent Bernoulli(p_j) over cols."""
    out: dict[frozenset, Fraction] = {}
    for bits in product((0, 1), repeat=len(cols)):
        w = Fraction(1)
        acc = []
        for j, bit in zip(cols, bits):
            w *= p[j] if bit else (1 - p[j])
            if bit:
                acc.append(j)
        if w:
            out[frozenset(acc)] = out.get(frozenset(acc), Fraction(0)) + w
    return out


def row_law(zs, r: int, segments, ys=None, Y=None, force_first: bool = False, chung_lu: bool = False):
    """Law of row r's accepted columns for sorted parameters zs (and ys).

    segments: list of (a, b) column ranges covering (r, N).
    ys is None: UBCM, or with chung_lu the Chung-Lu model (proposal = target
    in both).  Otherwise UECM with bound value Y (the Y used for row r).
    Returns (law, target_law).
    """
    n = len(zs)
    s = zs[r]
    p, qcol = {}, {}
    for j in range(r, n):
        t = s * zs[j]  # float product, as the sampler computes it
        if chung_lu:
            p[j] = chung_lu_p(t)
            qcol[j] = p[j]
        elif ys is None:
            p[j] = ubcm_p(t)
            qcol[j] = p[j]
        else:
            b = ys[r] * ys[j]
            p[j] = uecm_p(t, b)
            qcol[j] = uecm_bound(t, Y)
    law = {frozenset(): Fraction(1)}
    for (a, b) in segments:
        q_start = qcol[a - 1]
        law = combine(law, segment_law(p, qcol, a, b, q_start, force_first=force_first))
    cols = list(range(r + 1, n))
    return law, bernoulli_law(p, cols)


def top2_product(vals) -> float:
    v = sorted(vals, reverse=True)
    if len(v) < 2:
        return 0.0
    return v[0] * v[1]
