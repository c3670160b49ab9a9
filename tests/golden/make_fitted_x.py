"""Writes ubcm_fit_n1e6.txt: x fitted on the CPU to the N = 1,000,000
power-law targets (exponent 2.1, k in [1, 10^4], the seeded draw of
workloads.cfg2_degrees()), one value per degree class.

The fit is the fixed point x_c <- x_c k*_c / k_c(x) over degree classes
(nodes with equal targets share their parameter), with expected degrees
from the oracle's compensated sums with class multiplicities, stopped at a
relative residual of 1e-10.  Only the oracle computes here.  Each line:
target degree, class size, x as a hexadecimal float (exact round trip).

Usage: python tests/golden/make_fitted_x.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "ubcm_fit_n1e6.txt")
TOL = 1e-10


def fit_classes(k, tol=TOL, max_iter=20_000):
    kc, cnt = np.unique(np.asarray(k, np.float64), return_counts=True)
    m = cnt.astype(np.float64)
    x = kc / np.sqrt(np.sum(k))
    for it in range(1, max_iter + 1):
        kk, _ = oracle.expected_degree(x, None, m)
        res = float(np.max(np.abs(kk - kc) / kc))
        if res <= tol:
            return kc, cnt, x, it, res
        x = x * (kc / kk)
    raise RuntimeError("fixed point did not converge")


def main():
    k = workloads.cfg2_degrees()
    kc, cnt, x, it, res = fit_classes(k)
    with open(OUT, "w") as f:
        f.write("# x fitted to the N = 1,000,000 power-law targets (2.1 on [1, 10^4]); written by make_fitted_x.py\n")
        f.write(f"# fixed point over {len(kc)} degree classes, {it} iterations, relative residual {res:.3e}\n")
        f.write("# columns: target degree, nodes in the class, x (hexadecimal float)\n")
        for a, b, c in zip(kc, cnt, x):
            f.write(f"{int(a)} {int(b)} {float(c).hex()}\n")
    print(f"wrote {OUT}: {len(kc)} classes, {it} iterations, residual {res:.3e}")


if __name__ == "__main__":
    main()
