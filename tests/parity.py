"""Edge-list comparison shared by the GPU parity tests.

The bar (exactness of the method, Sec. 2.3: the sampler draws each pair with
its exact probability, so the GPU and the oracle, fed the same counters, draw
the same sample): the GPU edge list equals the oracle's edge for edge (and
weight for weight), except for edges of rows in which the oracle saw a
floating-point decision within 1e-12 of its threshold (its near-tie trace):
there the host and device logarithms, which may differ by a few ulp, can take
the decision either way.  Every edge present in one list and not the other,
or present in both with different weights, is a divergence.  Divergences must
lie in near-tie rows and number at most one per 1e7 edges compared (at least
one is allowed).  Each comparison is recorded in LEDGER, and the session's
totals are printed at its end (tests/conftest.py).
"""
from __future__ import annotations

import numpy as np

DIVERGENCES_PER_EDGE = 1e-7

# one entry per comparison: (label, divergences, edges compared, near-tie rows)
LEDGER: list = []


def allowed_divergences(edges_compared: int) -> int:
    return max(1, int(edges_compared * DIVERGENCES_PER_EDGE))


def edge_divergences(gs, gd, gw, os_, od, ow, n_cols: int, tie_rows, label: str = "") -> int:
    """Compares two edge lists (numpy arrays; gw/ow None when unweighted).

    Asserts: no pair twice in either list; every divergence in a row of the
    oracle's near-tie trace; at most allowed_divergences(len(oracle list)).
    Returns the number of divergences."""
    gk = np.asarray(gs, np.int64) * n_cols + np.asarray(gd, np.int64)
    ok = np.asarray(os_, np.int64) * n_cols + np.asarray(od, np.int64)
    og, oo = np.argsort(gk, kind="stable"), np.argsort(ok, kind="stable")
    gk, ok = gk[og], ok[oo]
    assert np.all(gk[1:] != gk[:-1]), f"{label}: a pair appears twice in the GPU list"
    assert np.all(ok[1:] != ok[:-1]), f"{label}: a pair appears twice in the oracle list"
    only_g = np.setdiff1d(gk, ok, assume_unique=True)
    only_o = np.setdiff1d(ok, gk, assume_unique=True)
    diff_keys = [only_g, only_o]
    if gw is not None:
        common, ig, io = np.intersect1d(gk, ok, assume_unique=True, return_indices=True)
        wg = np.asarray(gw)[og][ig]
        wo = np.asarray(ow)[oo][io]
        diff_keys.append(common[wg != wo])
    diff = np.concatenate(diff_keys)
    n_div = len(only_g) + len(only_o) + (len(diff_keys[2]) if gw is not None else 0)
    if n_div:
        rows = diff // n_cols
        outside = ~np.isin(rows, np.asarray(tie_rows, np.int64))
        assert not outside.any(), (
            f"{label}: {int(outside.sum())} of {n_div} differing edges lie outside the near-tie rows, "
            f"e.g. pair {int(diff[outside][0]) // n_cols} -> {int(diff[outside][0]) % n_cols}")
    compared = len(ok)
    LEDGER.append((label, n_div, compared, len(tie_rows)))
    assert n_div <= allowed_divergences(compared), (
        f"{label}: {n_div} divergences in {compared} edges (allowed {allowed_divergences(compared)})")
    return n_div


def summary() -> dict:
    return {"comparisons": len(LEDGER), "divergences": sum(e[1] for e in LEDGER),
            "edges_compared": sum(e[2] for e in LEDGER), "near_tie_rows": sum(e[3] for e in LEDGER)}
