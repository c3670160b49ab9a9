"""Maximum-likelihood fit of x (and y) to target degrees (and strengths).

The fit is not the paper's contribution (it uses an external solver, Sec. 3),
but the sampler needs fitted parameters.  Both fits run on the device through
the expected-degree kernel and its adjoint:

* unweighted: the fixed point x_c <- x_c k*_c / k_c(x) over degree classes
  (nodes with equal targets share their parameter), with class multiplicities
  passed to the forward kernel;
* weighted: Newton-CG on the convex negative log-likelihood in natural
  coordinates (log x, log y).  Its gradient is (k(x,y) - k*, s(x,y) - s*) and
  its Hessian-vector product is the adjoint of (k, s) applied to the vector,
  times (x, y) by the chain rule.

Residuals are reported as max_c |k_c - k*_c| / k*_c (and the same for s).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import expected_degree, expected_degree_grad


@dataclass
class FitResult:
    x: np.ndarray
    y: np.ndarray | None
    iterations: int
    residual: float
    residual_s: float | None = None


def _classes(*targets):
    key = np.stack([np.asarray(t, dtype=np.float64) for t in targets], axis=1)
    uniq, inverse, counts = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    return uniq, inverse.reshape(-1), counts.astype(np.float64)


def fit_ubcm(k_target, tol: float = 1e-10, max_iter: int = 20_000, device: str = "cuda") -> FitResult:
    """Fit x so that every node's expected degree matches k_target (all > 0)."""
    k_target = np.asarray(k_target, dtype=np.float64)
    if np.any(k_target <= 0):
        raise ValueError("target degrees must be positive")
    uniq, inv, m = _classes(k_target)
    kc = torch.as_tensor(uniq[:, 0], device=device)
    mult = torch.as_tensor(m, device=device)
    x = kc / float(np.sqrt(k_target.sum()))
    res = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        k, _ = expected_degree(x, None, mult)
        rel = torch.abs(k - kc) / kc
        if it % 16 == 1 or it == max_iter:
            res = float(rel.max())
            if res <= tol:
                break
        x = x * (kc / k)
    k, _ = expected_degree(x, None, mult)
    res = float((torch.abs(k - kc) / kc).max())
    return FitResult(x=x.cpu().numpy()[inv], y=None, iterations=it, residual=res)


def fit_uecm(k_target, s_target, tol: float = 1e-8, max_newton: int = 200, cg_iters: int = 100,
             device: str = "cuda", x0=None, y0=None, verbose: bool = False) -> FitResult:
    """Fit (x, y) so that expected degrees and strengths match the targets.

    Requires 0 < k_i <= s_i.  Nodes with s_i == k_i have no finite MLE (y -> 0,
    x -> infinity with x*y finite); they are held at y = 1e-12.
    """
    k_target = np.asarray(k_target, dtype=np.float64)
    s_target = np.asarray(s_target, dtype=np.float64)
    uniq, inv, m = _classes(k_target, s_target)
    kc = torch.as_tensor(uniq[:, 0], device=device)
    sc = torch.as_tensor(uniq[:, 1], device=device)
    mult = torch.as_tensor(m, device=device)
    degenerate = sc <= kc
    if x0 is None:
        yb = torch.sqrt(torch.clamp(1.0 - kc / sc, 1e-12, 0.999))
        z = kc / float(np.sqrt(k_target.sum()))
        x0 = z / yb
        y0 = yb
    else:
        x0 = torch.as_tensor(np.asarray(x0)[np.unique(inv, return_index=True)[1]], device=device)
        y0 = torch.as_tensor(np.asarray(y0)[np.unique(inv, return_index=True)[1]], device=device)
    th = torch.log(x0)
    et = torch.log(torch.clamp(y0, 1e-12, 0.999))
    free_y = ~degenerate

    def grad(th, et):
        x, y = torch.exp(th), torch.exp(et)
        k, s = expected_degree(x, y, mult)
        g1 = (k - kc) * mult
        g2 = torch.where(free_y, (s - sc) * mult, torch.zeros_like(s))
        return g1, g2, k, s

    def hvp(th, et, v1, v2):
        x, y = torch.exp(th), torch.exp(et)
        # Hessian of the class-compressed NLL: J^T diag(m) applied to (v1, v2) where
        # J = d(k, s)/d(log x, log y); the adjoint takes the upstream m * v.
        gx, gy = expected_degree_grad(x, y, mult, (mult * v1).contiguous(), (mult * v2).contiguous())
        h1 = gx * x
        h2 = torch.where(free_y, gy * y, torch.zeros_like(gy))
        return h1, h2

    res_k = res_s = np.inf
    it = 0
    for it in range(1, max_newton + 1):
        g1, g2, k, s = grad(th, et)
        res_k = float((torch.abs(k - kc) / kc).max())
        res_s = float((torch.abs(s - sc) / sc)[free_y].max()) if bool(free_y.any()) else 0.0
        if verbose:
            print(f"newton {it}: res_k={res_k:.3e} res_s={res_s:.3e}")
        if res_k <= tol and res_s <= tol:
            break
        # conjugate gradients on H d = -g
        d1 = torch.zeros_like(g1)
        d2 = torch.zeros_like(g2)
        r1, r2 = -g1, -g2
        p1, p2 = r1.clone(), r2.clone()
        rr = float((r1 * r1).sum() + (r2 * r2).sum())
        rr0 = rr
        for _ in range(cg_iters):
            h1, h2 = hvp(th, et, p1, p2)
            php = float((p1 * h1).sum() + (p2 * h2).sum())
            if php <= 0:
                break
            a = rr / php
            d1 += a * p1
            d2 += a * p2
            r1 -= a * h1
            r2 -= a * h2
            rr_new = float((r1 * r1).sum() + (r2 * r2).sum())
            if rr_new <= 1e-24 * rr0:
                break
            p1 = r1 + (rr_new / rr) * p1
            p2 = r2 + (rr_new / rr) * p2
            rr = rr_new
        # backtracking on feasibility (y_i y_j < 1) and gradient norm
        step = 1.0
        gn = float((g1 * g1).sum() + (g2 * g2).sum())
        for _ in range(30):
            th_n = th + step * d1
            et_n = torch.clamp(et + step * d2, max=-1e-12)
            ys = torch.sort(et_n, descending=True).values
            feasible = ys.numel() < 2 or float(ys[0] + ys[1]) < 0
            if feasible:
                n1, n2, _, _ = grad(th_n, et_n)
                if float((n1 * n1).sum() + (n2 * n2).sum()) < gn or step < 1e-6:
                    break
            step *= 0.5
        th, et = th_n, et_n
    x, y = torch.exp(th), torch.exp(et)
    return FitResult(x=x.cpu().numpy()[inv], y=y.cpu().numpy()[inv], iterations=it, residual=res_k, residual_s=res_s)
