"""The stored fitted parameters of the N = 1M workload (tests/golden/
ubcm_fit_n1e6.txt) are the oracle's fit: recomputed here and compared bit for
bit, and their expected degrees match the targets."""
import os
import sys

import numpy as np

import oracle
import workloads

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
import make_fitted_x  # noqa: E402


def test_stored_fit_is_the_oracle_fit():
    k = workloads.cfg2_degrees()
    kc, cnt, x, it, res = make_fitted_x.fit_classes(k)
    assert res <= 1e-10
    stored = workloads.cfg2_fitted_x()
    assert np.array_equal(stored, x[np.searchsorted(kc, k)])


def test_stored_fit_meets_targets():
    k = workloads.cfg2_degrees()
    kc, first, cnt = np.unique(k, return_index=True, return_counts=True)
    x = workloads.cfg2_fitted_x()[first]
    kk, _ = oracle.expected_degree(x, None, cnt.astype(np.float64))
    assert np.max(np.abs(kk - kc) / kc) <= 1e-10
