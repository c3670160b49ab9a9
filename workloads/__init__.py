"""Seeded synthetic inputs for the UBCM / UECM samplers.

This module is shared by the product path, the tests and the bench.  It holds
no arithmetic of the sampling method or of the models: it only draws node
parameters or target degree/strength sequences with the sizes and value
distributions of the workloads, from ``numpy.random.default_rng``.

The paper's evaluation networks (93 unweighted + 10 weighted empirical
networks, Sec. 3) are not available; these draws stand in for them.  Every
generator is a pure function of its arguments.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "powerlaw_degrees",
    "lognormal_x",
    "chung_lu_scale",
    "uecm_recipe",
    "cfg1_small",
    "cfg2_degrees",
    "cfg2_fitted_x",
    "cfg3_targets",
    "cfg4_networks",
    "cfg5_targets",
    "bipartite_params",
    "directed_params",
    "holme_kim",
    "sha256",
    "Network",
]


def sha256(a: np.ndarray) -> str:
    """Hex digest of an array's bytes (C order), logged next to each input."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def powerlaw_degrees(rng: np.random.Generator, n: int, gamma: float, kmin: int, kmax: int) -> np.ndarray:
    """Integer degrees drawn from P(k) proportional to k^-gamma on [kmin, kmax].

    Inverse-CDF sampling on the exact (truncated, discrete) pmf.
    """
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    pmf = ks ** (-gamma)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    u = rng.random(n)
    idx = np.searchsorted(cdf, u, side="right")
    idx = np.minimum(idx, len(ks) - 1)
    return (kmin + idx).astype(np.int64)


def lognormal_x(rng: np.random.Generator, n: int, mu: float, sigma: float) -> np.ndarray:
    """x_i = exp(z_i), z_i ~ Normal(mu, sigma)."""
    return np.exp(rng.normal(mu, sigma, size=n)).astype(np.float64)


def chung_lu_scale(k: np.ndarray) -> np.ndarray:
    """Starting parameters x_i = k_i / sqrt(sum k): the sparse-limit scaling.

    Used as a recipe for parameter vectors with the shape of a fitted
    power-law network, and as the starting point of a fit.
    """
    k = np.asarray(k, dtype=np.float64)
    return k / np.sqrt(k.sum())


def uecm_recipe(k: np.ndarray, s: np.ndarray, ymax: float = 0.999) -> tuple[np.ndarray, np.ndarray]:
    """(x, y) with the shape of fitted weighted parameters for targets (k, s).

    y_i = sqrt(1 - k_i/s_i) (mean weight per edge of about s/k), clipped to
    [0, ymax]; the product x_i*y_i follows the sparse-limit scaling of k.
    Nodes with s_i == k_i get y_i = 0 and x_i = 0 would follow, so they are
    given a tiny y and a large x whose product keeps that scaling.
    """
    k = np.asarray(k, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    y = np.sqrt(np.clip(1.0 - k / s, 0.0, 1.0))
    y = np.clip(y, 1e-6, ymax)
    z = k / np.sqrt(k.sum())
    x = z / y
    return x, y


@dataclass
class Network:
    """One network of a batched ensemble."""

    x: np.ndarray
    y: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def cfg1_small(seed: int = 1, n: int = 2000) -> np.ndarray:
    """Small unweighted case: x_i = exp(Normal(-4, 1.5)), N = 2,000."""
    rng = np.random.default_rng(seed)
    return lognormal_x(rng, n, -4.0, 1.5)


def cfg2_degrees(seed: int = 2, n: int = 1_000_000) -> np.ndarray:
    """Target degrees for the N = 1M unweighted case: power law 2.1 on [1, 10^4]."""
    rng = np.random.default_rng(seed)
    return powerlaw_degrees(rng, n, 2.1, 1, 10_000)


FITTED_X_CFG2 = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                             "ubcm_fit_n1e6.txt")


def cfg2_fitted_x(path: str = FITTED_X_CFG2) -> np.ndarray:
    """x for the N = 1M targets of cfg2_degrees(), one value per degree class,
    read from the stored CPU fit (tests/golden/make_fitted_x.py writes it):
    every node takes its class's value.  The class sizes are checked against
    the draw."""
    k = cfg2_degrees()
    table = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            deg, cnt, xh = line.split()
            table[int(deg)] = (int(cnt), float.fromhex(xh))
    kc, cnt = np.unique(k, return_counts=True)
    if len(kc) != len(table) or any(table.get(int(a), (-1,))[0] != int(b) for a, b in zip(kc, cnt)):
        raise ValueError(f"{path} does not match the degree classes of cfg2_degrees()")
    xc = np.array([table[int(a)][1] for a in kc], dtype=np.float64)
    return xc[np.searchsorted(kc, k)]


def cfg3_targets(seed: int = 3, n: int = 200_000) -> tuple[np.ndarray, np.ndarray]:
    """Weighted case targets: k ~ power law 2.3 on [1, 5000];
    s_i = round(k_i * (1 + Gamma(shape 2, scale 3)))."""
    rng = np.random.default_rng(seed)
    k = powerlaw_degrees(rng, n, 2.3, 1, 5_000)
    g = rng.gamma(2.0, 3.0, size=n)
    s = np.rint(k * (1.0 + g)).astype(np.int64)
    s = np.maximum(s, k)
    return k, s


def cfg4_networks(seed: int = 4, n_networks: int = 256, nmin: float = 1e3, nmax: float = 2e5) -> list[Network]:
    """Batched ensemble: N_n = round(exp(Uniform(ln nmin, ln nmax))),
    x = exp(Normal(-5, 2)) per network."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=n_networks))).astype(np.int64)
    nets = []
    for i, n in enumerate(sizes):
        nets.append(Network(x=lognormal_x(rng, int(n), -5.0, 2.0), meta={"index": i, "n": int(n)}))
    return nets


def cfg5_targets(seed: int = 5, n_ubcm: int = 100_000, n_uecm: int = 50_000, kmax: int = 2_000):
    """Fit-then-sample case: UBCM degrees power law 2.5 on [2, kmax];
    UECM targets drawn like the weighted case."""
    rng = np.random.default_rng(seed)
    k_u = powerlaw_degrees(rng, n_ubcm, 2.5, 2, kmax)
    k_w = powerlaw_degrees(rng, n_uecm, 2.3, 1, 5_000)
    g = rng.gamma(2.0, 3.0, size=n_uecm)
    s_w = np.maximum(np.rint(k_w * (1.0 + g)).astype(np.int64), k_w)
    return k_u, (k_w, s_w)


def bipartite_params(seed: int = 6, n_rows: int = 1_000_000, n_cols: int = 500_000, weighted: bool = False):
    """Two-set case (Sec. 2.6): row degrees power law 2.1 on [1, 10^4], column
    degrees power law 2.5 on [1, 10^4] rescaled to the same edge total;
    x+ = k+ / sqrt(E), x- = k- / sqrt(E) (E = sum of row degrees), the
    sparse-limit scaling of a bipartite network.  Weighted: y+ and y- uniform
    on [0.05, 0.95]; the product z = x y keeps that scaling.
    Returns (x_rows, x_cols, y_rows, y_cols) with y None when unweighted."""
    rng = np.random.default_rng(seed)
    kr = powerlaw_degrees(rng, n_rows, 2.1, 1, 10_000).astype(np.float64)
    kc = powerlaw_degrees(rng, n_cols, 2.5, 1, 10_000).astype(np.float64)
    kc *= kr.sum() / kc.sum()
    e = np.sqrt(kr.sum())
    zr, zc = kr / e, kc / e
    if not weighted:
        return zr, zc, None, None
    yr = rng.uniform(0.05, 0.95, n_rows)
    yc = rng.uniform(0.05, 0.95, n_cols)
    return zr / yr, zc / yc, yr, yc


def directed_params(seed: int = 7, n: int = 500_000, weighted: bool = False):
    """Directed case (Sec. 2.6): out- and in-degrees, power laws 2.2 and 2.6 on
    [1, 5000], drawn independently, in-degrees rescaled to the out total;
    x_out = k_out / sqrt(E), x_in = k_in / sqrt(E).  Weighted: y uniform on
    [0.05, 0.95] for each side.  Returns (x_out, x_in, y_out, y_in)."""
    rng = np.random.default_rng(seed)
    ko = powerlaw_degrees(rng, n, 2.2, 1, 5_000).astype(np.float64)
    ki = powerlaw_degrees(rng, n, 2.6, 1, 5_000).astype(np.float64)
    ki *= ko.sum() / ki.sum()
    e = np.sqrt(ko.sum())
    if not weighted:
        return ko / e, ki / e, None, None
    yo = rng.uniform(0.05, 0.95, n)
    yi = rng.uniform(0.05, 0.95, n)
    return ko / e / yo, ki / e / yi, yo, yi


def holme_kim(n: int = 5000, m: int = 10, p_triad: float = 0.1, seed: int = 8) -> tuple[np.ndarray, np.ndarray]:
    """Edge list (src, dst; each edge once, src < dst) of a Holme-Kim network
    (Holme and Kim, Phys. Rev. E 65, 026107, 2002): growth by preferential
    attachment with triad formation, the clustered power-law network of the
    paper's Fig. 1 (5,000 nodes, m = 10, triad probability 0.1).

    The first m nodes start without edges and node m links to all of them.
    Each later node v makes m links: the first to a node drawn with
    probability proportional to its degree; each further one, with probability
    p_triad, to a random neighbour of the node of the previous preferential
    link that v is not yet linked to (if there is one), and otherwise again by
    preferential attachment.  No multi-edges, no self-loops."""
    rng = np.random.default_rng(seed)
    ends: list[int] = []  # every edge's two ends: a uniform draw is a degree-proportional one
    nbr: list[list[int]] = [[] for _ in range(n)]
    src, dst = [], []

    def pref(v, linked):
        # at least m + 1 nodes have edges once node m has linked, and v is
        # linked to at most m - 1 of them: the draw ends
        while True:
            u = int(ends[rng.integers(len(ends))])
            if u != v and u not in linked:
                return u

    def link(u, v):
        nbr[u].append(v)
        nbr[v].append(u)
        ends.extend((u, v))
        src.append(min(u, v))
        dst.append(max(u, v))

    for u in range(min(m, n - 1)):
        link(u, m)
    for v in range(m + 1, n):
        linked: set[int] = set()
        last_pref = None
        for k in range(m):
            u = None
            if k > 0 and last_pref is not None and rng.random() < p_triad:
                cand = [w for w in nbr[last_pref] if w != v and w not in linked]
                if cand:
                    u = cand[int(rng.integers(len(cand)))]
            if u is None:
                u = pref(v, linked)
                last_pref = u
            linked.add(u)
            link(u, v)
    return np.asarray(src, dtype=np.int32), np.asarray(dst, dtype=np.int32)
