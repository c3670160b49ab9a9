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
  times (x, y) by the chain rule.  CG is Jacobi-preconditioned with the
  leading diagonal terms (m k, m s); the step length comes from the sign of
  the directional derivative along the Newton direction (the objective is
  convex), bisected when the full step overshoots.

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
    x -> infinity with x*y finite); their y is held at its start, 1e-6, and only
    x is fitted for them (their strength then exceeds k_i by a relative ~1e-6).
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

    # The model needs y_i y_j < 1 for every pair of distinct nodes: the two
    # largest y multiply below 1, and a class of several nodes (paired with
    # itself) keeps y < 1; a class of one node may have y > 1.  (Its own pair
    # has weight zero; the kernels still evaluate it, with b = y^2 > 1, and its
    # terms stay finite unless 1 - b + ab is exactly 0.)
    multi = mult >= 2

    def feasible(et_n):
        top = torch.topk(et_n, 2).values if et_n.numel() >= 2 else et_n
        ok = et_n.numel() < 2 or float(top[0] + top[1]) < 0
        return ok and not bool((et_n[multi] >= 0).any())

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
        # preconditioned conjugate gradients on H d = -g; Jacobi scale from the
        # diagonal's leading terms (m k for log x, m s for log y)
        P1 = 1.0 / torch.clamp(mult * k, min=1e-300)
        P2 = torch.where(free_y, 1.0 / torch.clamp(mult * s, min=1e-300), torch.zeros_like(s))
        d1 = torch.zeros_like(g1)
        d2 = torch.zeros_like(g2)
        r1, r2 = -g1, -g2
        z1, z2 = P1 * r1, P2 * r2
        p1, p2 = z1.clone(), z2.clone()
        rz = float((r1 * z1).sum() + (r2 * z2).sum())
        rz0 = rz
        for _ in range(cg_iters):
            h1, h2 = hvp(th, et, p1, p2)
            php = float((p1 * h1).sum() + (p2 * h2).sum())
            if php <= 0:
                break
            a = rz / php
            d1 += a * p1
            d2 += a * p2
            r1 -= a * h1
            r2 -= a * h2
            z1, z2 = P1 * r1, P2 * r2
            rz_new = float((r1 * z1).sum() + (r2 * z2).sum())
            if rz_new <= 1e-28 * rz0:
                break
            p1 = z1 + (rz_new / rz) * p1
            p2 = z2 + (rz_new / rz) * p2
            rz = rz_new
        # line search on the directional derivative phi'(t) = d . grad(theta + t d) (convex):
        # keep t = 1 while phi' < 0 there, else bisect for phi' = 0 on [0, 1]
        def dphi(t):
            et_n = torch.where(multi, torch.clamp(et + t * d2, max=-1e-12), et + t * d2)
            if not feasible(et_n):
                return None, None, None
            n1, n2, _, _ = grad(th + t * d1, et_n)
            return float((d1 * n1).sum() + (d2 * n2).sum()), th + t * d1, et_n

        t_hi = 1.0
        val, th_n, et_n = dphi(t_hi)
        while val is None and t_hi > 1e-8:
            t_hi *= 0.5
            val, th_n, et_n = dphi(t_hi)
        if val is None:
            break
        if val > 0:
            lo, hi = 0.0, t_hi
            for _ in range(12):
                mid = 0.5 * (lo + hi)
                v, th_m, et_m = dphi(mid)
                if v is None or v > 0:
                    hi = mid
                else:
                    lo, th_n, et_n = mid, th_m, et_m
            if lo == 0.0:
                _, th_n, et_n = dphi(hi)
        th, et = th_n, et_n
    x, y = torch.exp(th), torch.exp(et)
    return FitResult(x=x.cpu().numpy()[inv], y=y.cpu().numpy()[inv], iterations=it, residual=res_k, residual_s=res_s)
