#!/usr/bin/env python3
"""Throughput of the MI355X sampler on the N = 1,000,000 unweighted workload.

One step = one full sample: node order (radix sort), plan, segmented sweep
with edge compaction, on parameters already resident in HBM.  Target degrees
follow a discrete power law (exponent 2.1, k in [1, 10^4]) and x is fitted to
them on the device (untimed).  Every step draws a new replica (a new sample).
The timed samples are issued back to back on one stream through the
asynchronous entry point (no host round trip between samples) and the clock
stops after the stream has drained; their edge counts come from an untimed
repeat of the same samples, which are identical (counter-based randomness; the
last one is checked against the timed run's own count).  The timed samples
record events only around the sweep; the order and plan stage times come from
the repeat.

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sampled edges/s (unweighted, N=1M) + replicas/s batched vs plain, same GPU"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes per cycle at 2.4 GHz (one VALU instruction
# of a 64-wide wave issues over 4 cycles): 39.3e12 lane-operations/s for
# full-rate 32-bit integer and binary64 vector instructions.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0

# VALU instructions of one step of the sweep on its common path, counted in the
# gfx950 code of k_sweep<false,false>: the draw (Philox block, the two
# uniforms, the log of U1) 93, the acceptance test 15, the skip (log1p, the
# division, the next candidate's address) 67, the candidate load 1; loop,
# refill and staging instructions are not counted as work.
SWEEP_VALU_PER_STEP = 176

# HBM bytes of one unweighted k_sweep launch on the timed workload (stored fit,
# seg_work 8), from two rocprofv3 --pmc runs: FETCH_SIZE and WRITE_SIZE in KiB
# per dispatch (medians over the timed samples), scaled by what the same
# counters read for a 256 MiB copy (fetched bytes = 2 x FETCH_SIZE, written =
# 1 x WRITE_SIZE).  They hold for the sweep built from the sources hashed in
# SWEEP_SOURCES only; for any other build or input the bench reports null.
SWEEP_COUNTERS = {"fetch_kib": 107300, "write_kib": 16366, "fetch_scale": 2.0, "write_scale": 1.0,
                  "sources_sha256": "369d7138187e68df5636896cbf79f7f604a5aefa97c62fa74cf18adb8134a247",
                  "input_sha256": "bc9851eaa93191638377524467d37dbbae5a37d6523e29d9c327d955e13c3ef6",
                  "seg_work": 8}
SWEEP_SOURCES = ["paper_2509_13230_amd/csrc/" + f for f in
                 ("mh_sweep.hip", "mh_sweep_core.hpp", "mh_stage.hpp", "mh_common.hpp", "mh_prepare.hpp",
                  "mh_internal.hpp", "mh_lookback.hpp")] + ["include/mh.h"]


def sweep_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


class HipEvents:
    """Timing events without the system-scope fence at record time (the stream
    is synchronised before they are read), so that recording one does not
    write back and invalidate the caches between the kernels it separates."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self, n: int, present=None):
        """n slots; present(i) false leaves slot i NULL (a stage not timed)."""
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreateWithFlags.argtypes = [ctypes.c_void_p, ctypes.c_uint]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * n)()
        for i in range(n):
            if present is not None and not present(i):
                continue
            ev = ctypes.c_void_p()
            rc = self.rt.hipEventCreateWithFlags(ctypes.byref(ev), self.DISABLE_SYSTEM_FENCE)
            if rc != 0:
                raise RuntimeError("hipEventCreateWithFlags failed")
            self.arr[i] = ev.value

    @property
    def address(self) -> int:
        return ctypes.addressof(self.arr)

    def elapsed_ms(self, a: int, b: int) -> float:
        self.rt.hipEventSynchronize(self.arr[b])
        out = ctypes.c_float(0)
        rc = self.rt.hipEventElapsedTime(ctypes.byref(out), self.arr[a], self.arr[b])
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)


def edge_divergences(gs, gd, os_, od, n: int, tie_rows) -> tuple[int, int]:
    """(divergences, of which outside near-tie rows) between a GPU and an
    oracle edge list of one sample: pairs present in one list only."""
    gk = np.sort(np.asarray(gs, np.int64) * n + np.asarray(gd, np.int64))
    ok = np.sort(np.asarray(os_, np.int64) * n + np.asarray(od, np.int64))
    diff = np.concatenate([np.setdiff1d(gk, ok, assume_unique=True), np.setdiff1d(ok, gk, assume_unique=True)])
    outside = int((~np.isin(diff // n, np.asarray(tie_rows, np.int64))).sum()) if len(diff) else 0
    return len(diff), outside


def cpu_baseline(x: np.ndarray, seed: int, seg_work: int, budget_s: float, replicas: list, gpu_sample) -> dict:
    """The CPU oracle (sequential, one thread) on whole samples of the same
    workload and the same (seed, replica) pairs as the timed samples.  After
    the clock, each oracle sample is compared with the GPU's sample of the same
    replica (gpu_sample(replica) -> (src, dst) numpy arrays), edge for edge."""
    import oracle

    oracle.build()
    t_total = 0.0
    edges = 0
    reps = 0
    samples = []
    while reps < 1 or (t_total < budget_s and reps < len(replicas)):
        t0 = time.perf_counter()
        s = oracle.sample_mh(x, None, seed=seed, replica=replicas[reps], seg_work=seg_work, capacity=int(2.5e6))
        t_total += time.perf_counter() - t0
        edges += s.n_edges
        samples.append((replicas[reps], s))
        reps += 1
    n = len(x)
    div = outside = ties = 0
    for r, s in samples:
        gs, gd = gpu_sample(r)
        d, o = edge_divergences(gs, gd, s.src, s.dst, n, s.tie_rows)
        div += d
        outside += o
        ties += len(s.tie_rows)
    try:
        host_cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        host_cpus = os.cpu_count()
    return {"value": edges / t_total, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "host_cpus": host_cpus,
            "sample": f"{reps} whole samples of the N=1M workload (order + plan + sequential sweep), the timed "
                      f"samples' (seed, replica) pairs first, {t_total:.1f} s single-threaded",
            "parity": {"samples_compared": reps, "edges_compared": edges, "divergences": div,
                       "divergences_outside_near_tie_rows": outside, "near_tie_rows": ties,
                       "allowed": max(1, int(edges * 1e-7))}}


def small_bench(args, dev) -> dict:
    """The N = 2,000 network (x = exp(Normal(-4, 1.5))): microseconds per
    sample of the plain MH sampler and of the GPU brute force, as synchronous
    calls (each reads its edge count back; the best of many), and of MH
    samples issued back to back through the asynchronous entry point."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads

    xn = workloads.cfg1_small(seed=1)
    x = torch.as_tensor(xn, device=dev)
    n = x.numel()
    L = mh.lib()
    plan = mh.PlanParams(args.seg_work, 0, 0, 0, None)
    ws = torch.empty(L.mh_workspace_bytes(n, 0, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    src = torch.empty(64 * n, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)

    def best(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return min(t), out

    t_mh, (sm, _) = best(lambda: mh.sample_unweighted(x, seed=args.seed, replica=0, seg_work=args.seg_work,
                                                      out=(src, dst), workspace=ws), 50)
    t_bf, (sb, _) = best(lambda: mh.sample_bruteforce(x, seed=args.seed, replica=0, out=(src, dst)), 50)
    k = 200
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(k):
        mh.sample_async(x, None, (src, dst), ws, seed=args.seed, replica=r, seg_work=args.seg_work)
    torch.cuda.synchronize()
    t_async = (time.perf_counter() - t0) / k
    return {"workload": f"N={n}, x = exp(Normal(-4, 1.5)), one sample", "input_sha256": workloads.sha256(xn),
            "us_per_sample_mh_sync": t_mh * 1e6, "us_per_sample_mh_back_to_back": t_async * 1e6,
            "us_per_sample_bruteforce_sync": t_bf * 1e6, "edges_mh": int(sm.numel()), "edges_bruteforce": int(sb.numel()),
            "pairs": n * (n - 1) // 2}


# VALU instructions per pair of the brute-force sampler's loop (Philox block,
# the column's z, the uniform and the test), counted in the gfx950 code of
# k_bruteforce<false> (the Philox rounds' three-input xors one v_bitop3_b32
# each); staging of accepted pairs is not counted as work.
BF_VALU_PER_PAIR = 51


def bruteforce_vs_mh(args, x, dev) -> dict:
    """The GPU brute-force sampler (every pair with its own Philox block)
    against the plain MH sampler on one network: the first 50,000 nodes of the
    N = 1M workload with their fitted x.  Both are synchronous calls that read
    their edge count back; the time of each is the best of a few runs."""
    import torch

    import paper_2509_13230_amd as mh

    xp = x[: args.bf_prefix].contiguous()
    n = xp.numel()
    pairs = n * (n - 1) // 2

    def best(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return min(t), out

    t_bf, (sb, _) = best(lambda: mh.sample_bruteforce(xp, seed=args.seed, replica=0), 3)
    t_mh, (sm, _) = best(lambda: mh.sample_unweighted(xp, seed=args.seed, replica=0, seg_work=args.seg_work), 10)
    acc = degree_accuracy(args, xp, dev)
    return {
        "workload": f"first {n} nodes of the N=1M workload (their fitted x), one sample",
        "pairs": pairs,
        "ms_bruteforce": t_bf * 1e3,
        "pairs_per_s_bruteforce": pairs / t_bf,
        "edges_bruteforce": int(sb.numel()),
        "edges_per_s_bruteforce": sb.numel() / t_bf,
        "bruteforce_valu": {"achieved": pairs * BF_VALU_PER_PAIR / t_bf / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                            "unit": "TOP/s", "frac": pairs * BF_VALU_PER_PAIR / t_bf / PEAK_LANE_OPS},
        "ms_mh": t_mh * 1e3,
        "edges_mh": int(sm.numel()),
        "edges_per_s_mh": sm.numel() / t_mh,
        "speedup_mh_vs_bruteforce": t_bf / t_mh,
        "degree_accuracy": acc,
    }


def degree_accuracy(args, xp, dev) -> dict:
    """Both samplers' mean degrees over R replicas against the exact expected
    degrees: z_i = (mean_i - E_i) / sqrt(V_i / R), E_i = sum_j p_ij and
    V_i = sum_j p_ij (1 - p_ij) computed in float64 by torch over all pairs.
    An exact sampler gives z close to standard normal: |z| <= 4 for all but a
    few in 1e4 nodes and mean z^2 near 1."""
    import torch

    import paper_2509_13230_amd as mh

    n = xp.numel()
    R = args.accuracy_replicas
    E = torch.zeros(n, dtype=torch.float64, device=dev)
    V = torch.zeros(n, dtype=torch.float64, device=dev)
    for a in range(0, n, 2048):
        t = xp[a:a + 2048, None] * xp[None, :]
        p = t / (1.0 + t)
        idx = torch.arange(a, min(a + 2048, n), device=dev)
        p[idx - a, idx] = 0.0
        E[a:a + 2048] = p.sum(1)
        V[a:a + 2048] = (p * (1.0 - p)).sum(1)
    out = {"replicas": R, "nodes": n}
    for name, fn in (("mh", lambda r: mh.sample_unweighted(xp, seed=args.seed, replica=r, seg_work=args.seg_work)),
                     ("bruteforce", lambda r: mh.sample_bruteforce(xp, seed=args.seed, replica=r))):
        deg = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(R):
            s_, d_ = fn(100 + r)
            deg += torch.bincount(s_.long(), minlength=n).double() + torch.bincount(d_.long(), minlength=n).double()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        z = (deg / R - E) / torch.sqrt(V / R)
        out[name] = {"within_4_sigma": float((z.abs() <= 4).double().mean()), "max_abs_z": float(z.abs().max()),
                     "mean_z2": float((z * z).mean()), "ms_per_replica_incl_degree_count": el / R * 1e3}
    return out


# VALU instructions per (row, column) pair of the expected-degree kernels'
# inner loops, weighted, counted in their gfx950 code (one refined reciprocal
# per pair; per iteration of four pairs: forward 95, adjoint 148).
DEG_FWD_VALU_PER_PAIR = 95 / 4
DEG_BWD_VALU_PER_PAIR = 148 / 4


def expected_degree_bench(args, dev) -> dict:
    """The O(N^2) expected degree / strength reduction and its adjoint on the
    weighted N = 200,000 workload (power-law degrees 2.3 on [1, 5000], strengths
    k (1 + Gamma(2, 3)); parameters from the sparse-limit recipe)."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads

    k, st = workloads.cfg3_targets(seed=3, n=args.deg_n)
    xn, yn = workloads.uecm_recipe(k, st)
    x = torch.as_tensor(xn, device=dev)
    y = torch.as_tensor(yn, device=dev)
    n = x.numel()
    gk = torch.ones(n, dtype=torch.float64, device=dev)
    gs = torch.ones(n, dtype=torch.float64, device=dev)

    def best(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return min(t)

    t_f = best(lambda: mh.expected_degree(x, y))
    t_b = best(lambda: mh.expected_degree_grad(x, y, None, gk, gs))
    pairs = n * n
    return {
        "workload": f"UECM N={n}: forward (k, s) and adjoint (gx, gy), binary64",
        "pairs": pairs,
        "ms_forward": t_f * 1e3,
        "ms_adjoint": t_b * 1e3,
        "forward_valu": {"achieved": pairs * DEG_FWD_VALU_PER_PAIR / t_f / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "TOP/s", "frac": pairs * DEG_FWD_VALU_PER_PAIR / t_f / PEAK_LANE_OPS},
        "adjoint_valu": {"achieved": pairs * DEG_BWD_VALU_PER_PAIR / t_b / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "TOP/s", "frac": pairs * DEG_BWD_VALU_PER_PAIR / t_b / PEAK_LANE_OPS},
    }


def weighted_bench(args, dev, fitted: bool = False) -> dict:
    """The weighted sampler on the UECM N = 200,000 workload (power-law degrees
    2.3 on [1, 5000], strengths k (1 + Gamma(2, 3))): samples issued back to
    back on one stream, edges/s, and the stage times (order, bound + plan,
    sweep) of an untimed repeat.  Parameters from the sparse-limit recipe, or
    (fitted) from the device fit of the targets (Newton-CG on the likelihood,
    untimed; its residuals are reported)."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads
    from paper_2509_13230_amd.fit import fit_uecm

    k, st = workloads.cfg3_targets(seed=3, n=args.w_n)
    fit_info = None
    if fitted:
        t0 = time.perf_counter()
        f = fit_uecm(k, st, tol=1e-8, max_newton=args.w_fit_newton)
        fit_info = {"iterations": f.iterations, "residual_k": f.residual, "residual_s": f.residual_s,
                    "seconds": time.perf_counter() - t0, "y_max": float(f.y.max()),
                    "y_above_0.999": int((f.y > 0.999).sum())}
        xn, yn = f.x, f.y
    else:
        xn, yn = workloads.uecm_recipe(k, st)
    x = torch.as_tensor(xn, device=dev)
    y = torch.as_tensor(yn, device=dev)
    n = x.numel()
    L = mh.lib()
    plan = mh.PlanParams(args.w_seg_work, 0, 0, 0, None)
    ws = torch.empty(L.mh_workspace_bytes(n, 1, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    s0, _, _ = mh.sample_weighted(x, y, seed=args.seed, replica=0, seg_work=args.w_seg_work, workspace=ws)
    cap = int(len(s0) * 1.1) + 65536
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    w = torch.empty(cap, dtype=torch.int32, device=dev)
    steps = args.steps
    for i in range(args.warmup):
        mh.sample_async(x, y, (src, dst, w), ws, seed=args.seed, replica=1 + i, seg_work=args.w_seg_work)
    torch.cuda.synchronize()
    replicas = [3000 + i for i in range(steps)]
    t0 = time.perf_counter()
    for r in replicas:
        mh.sample_async(x, y, (src, dst, w), ws, seed=args.seed, replica=r, seg_work=args.w_seg_work)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last_edges = mh.sample_result(ws, cap)
    ev = HipEvents(4 * steps)
    ev_size = ctypes.sizeof(ctypes.c_void_p)
    edges = 0
    weight_sum = 0
    wsteps = 0
    wprops = 0
    stage = np.zeros(3)
    for i, r in enumerate(replicas):
        s_, _, w_, stt = mh.sample_weighted(x, y, seed=args.seed, replica=r, seg_work=args.w_seg_work, stats=True,
                                            out=(src, dst, w), workspace=ws,
                                            stage_events=ev.address + 4 * i * ev_size)
        stage += [ev.elapsed_ms(4 * i, 4 * i + 1), ev.elapsed_ms(4 * i + 1, 4 * i + 2),
                  ev.elapsed_ms(4 * i + 2, 4 * i + 3)]
        edges += stt["n_edges"]
        wsteps += stt["steps"]
        wprops += stt["proposals"]
        weight_sum += int(w_.sum().item())
    if stt["n_edges"] != last_edges:
        raise RuntimeError(f"timed and repeated weighted sample differ: {last_edges} vs {stt['n_edges']} edges")
    return {
        "workload": f"UECM N={n}, power-law degrees (exponent 2.3, k in [1, 5000]), strengths k (1 + Gamma(2, 3)), "
                    + ("parameters from the device fit of these targets" if fitted else "sparse-limit parameters")
                    + "; samples issued back to back on one stream",
        "fit": fit_info,
        "proposals_per_edge": wprops / max(edges, 1),
        "samples": steps,
        "seg_work": args.w_seg_work,
        "ms_per_sample": elapsed / steps * 1e3,
        "edges_per_s": edges / elapsed,
        "mean_edges_per_sample": edges / steps,
        "mean_weight": weight_sum / max(edges, 1),
        "steps_per_sample": wsteps / steps,
        "proposals_per_sample": wprops / steps,
        "stages_ms": {"order": stage[0] / steps, "bound_plan": stage[1] / steps, "sweep": stage[2] / steps},
    }


def bipartite_bench(args, dev) -> dict:
    """The two-set sampler (Sec. 2.6) on 1,000,000 rows (degrees power law 2.1
    on [1, 10^4]) x 500,000 columns (2.5, rescaled to the same edge total),
    sparse-limit parameters: synchronous samples (each reads its edge count
    back), edges/s and the stage times of the same calls."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads

    xr_n, xc_n, _, _ = workloads.bipartite_params(n_rows=args.bip_rows, n_cols=args.bip_rows // 2)
    xr = torch.as_tensor(xr_n, device=dev)
    xc = torch.as_tensor(xc_n, device=dev)
    L = mh.lib()
    plan = mh.PlanParams(args.bip_seg_work, 0, 0, 0, None)
    ws = torch.empty(L.mh_bipartite_workspace_bytes(xr.numel(), xc.numel(), 0, ctypes.byref(plan)),
                     dtype=torch.uint8, device=dev)
    first = mh.sample_bipartite(xr, xc, seed=args.seed, replica=0, seg_work=args.bip_seg_work, workspace=ws)
    cap = int(first.src.numel() * 1.1) + 65536
    out = (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev))
    for i in range(args.warmup):
        mh.sample_bipartite(xr, xc, seed=args.seed, replica=1 + i, seg_work=args.bip_seg_work, out=out, workspace=ws)
    steps = args.steps
    ev = HipEvents(4 * steps)
    ev_size = ctypes.sizeof(ctypes.c_void_p)
    edges = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        r = mh.sample_bipartite(xr, xc, seed=args.seed, replica=4000 + i, seg_work=args.bip_seg_work, out=out,
                                workspace=ws)
        edges += r.src.numel()
    elapsed = time.perf_counter() - t0
    # stage times from a repeat of the same samples with events (untimed)
    stage = np.zeros(3)
    for i in range(steps):
        mh.sample_bipartite(xr, xc, seed=args.seed, replica=4000 + i, seg_work=args.bip_seg_work, out=out,
                            workspace=ws, stage_events=ev.address + 4 * i * ev_size)
        stage += [ev.elapsed_ms(4 * i, 4 * i + 1), ev.elapsed_ms(4 * i + 1, 4 * i + 2),
                  ev.elapsed_ms(4 * i + 2, 4 * i + 3)]
    return {
        "workload": f"bipartite {xr.numel()} x {xc.numel()}, degrees power law 2.1 / 2.5 on [1, 10^4], sparse-limit "
                    "parameters; synchronous samples (edge count read back each time)",
        "samples": steps,
        "seg_work": args.bip_seg_work,
        "ms_per_sample": elapsed / steps * 1e3,
        "edges_per_s": edges / elapsed,
        "mean_edges_per_sample": edges / steps,
        "stages_ms": {"order": stage[0] / steps, "bound_plan": stage[1] / steps, "sweep": stage[2] / steps},
    }


def chung_lu_bench(args, dev) -> dict:
    """The Chung-Lu comparison model (Sec. 2.1, 2.3) and its bias.

    Speed: the Chung-Lu sampler on the N = 1M degrees (w = k / sqrt(2M)),
    samples back to back; the rank-count sink and the triangle count of those
    samples.  Bias (Fig. 1): a Holme-Kim network (5,000 nodes, m = 10, triad
    probability 0.1) gives the degrees; R samples of the Chung-Lu model and of
    the unbiased model fitted to the same degrees (device fit) are reduced to
    the density of edges among the top alpha of nodes and to triangle counts."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads
    from paper_2509_13230_amd.fit import fit_ubcm

    k = workloads.cfg2_degrees(seed=2, n=args.n).astype(np.float64)
    w = torch.as_tensor(k / np.sqrt(k.sum()), device=dev)
    n = w.numel()
    L = mh.lib()
    plan = mh.PlanParams(args.seg_work, 0, 0, 0, None)
    ws = torch.empty(L.mh_workspace_bytes(n, 0, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    s0, _ = mh.sample_chung_lu(w, seed=args.seed, replica=0, seg_work=args.seg_work, workspace=ws)
    cap = int(s0.numel() * 1.1) + 65536
    out = (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev))
    reps = 10
    for r in range(2):
        mh.sample_chung_lu(w, seed=args.seed, replica=r, seg_work=args.seg_work, out=out, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges = 0
    for r in range(reps):
        s_, _ = mh.sample_chung_lu(w, seed=args.seed, replica=2000 + r, seg_work=args.seg_work, out=out, workspace=ws)
        edges += s_.numel()
    torch.cuda.synchronize()
    t_cl = (time.perf_counter() - t0) / reps
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    t0 = time.perf_counter()
    for r in range(reps):
        mh.rank_counts(w, model=mh.MH_MODEL_CHUNG_LU, seed=args.seed, replica=2000 + r, seg_work=args.seg_work,
                       out=cnt, workspace=ws)
    torch.cuda.synchronize()
    t_rank = (time.perf_counter() - t0) / reps
    s_, d_ = mh.sample_chung_lu(w, seed=args.seed, replica=2000, seg_work=args.seg_work, out=out, workspace=ws)
    tws = torch.empty(L.mh_triangles_workspace_bytes(n, s_.numel()), dtype=torch.uint8, device=dev)
    mh.count_triangles(s_, d_, n, workspace=tws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tri_big = mh.count_triangles(s_, d_, n, workspace=tws)
    t_tri = time.perf_counter() - t0

    # the bias on Holme-Kim degrees
    hs, hd = workloads.holme_kim()
    hn = 5000
    hk = (np.bincount(hs, minlength=hn) + np.bincount(hd, minlength=hn)).astype(np.float64)
    hw = torch.as_tensor(hk / np.sqrt(hk.sum()), device=dev)
    fit = fit_ubcm(hk, tol=1e-10)
    hx = torch.as_tensor(fit.x, device=dev)
    order = np.argsort(-hk, kind="stable")
    alphas = [0.005, 0.01, 0.02, 0.05, 0.1]
    sizes = [max(2, int(round(a * hn))) for a in alphas]

    def density(c_np):
        cs = np.cumsum(c_np)
        return [float(cs[K - 1]) / (K * (K - 1) / 2) for K in sizes]

    rank_hk = np.empty(hn, dtype=np.int64)
    rank_hk[order] = np.arange(hn)
    hk_hi = np.maximum(rank_hk[hs], rank_hk[hd])
    hk_counts = np.bincount(hk_hi, minlength=hn)
    R = args.bias_replicas
    stats = {}
    hws = torch.empty(L.mh_workspace_bytes(hn, 0, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    htw = torch.empty(L.mh_triangles_workspace_bytes(hn, 4 * len(hs)), dtype=torch.uint8, device=dev)
    for name, par, model, sampler in (("chung_lu", hw, mh.MH_MODEL_CHUNG_LU, mh.sample_chung_lu),
                                      ("ubcm", hx, mh.MH_MODEL_UBCM, mh.sample_unweighted)):
        dens, tris, ms = [], [], []
        for r in range(R):
            c, m_ = mh.rank_counts(par, model=model, seed=args.seed, replica=r, seg_work=args.seg_work, workspace=hws)
            dens.append(density(c.cpu().numpy()))
            src_, dst_ = sampler(par, seed=args.seed, replica=r, seg_work=args.seg_work, workspace=hws)
            tris.append(mh.count_triangles(src_, dst_, hn, workspace=htw))
            ms.append(m_)
        dens = np.array(dens)
        stats[name] = {"rich_club_density": {f"{a:g}": [float(dens[:, i].mean()), float(dens[:, i].std())]
                                             for i, a in enumerate(alphas)},
                       "triangles": [float(np.mean(tris)), float(np.std(tris))],
                       "edges": [float(np.mean(ms)), float(np.std(ms))]}
    return {
        "workload": f"Chung-Lu model on the N={n} power-law degrees (w = k / sqrt(2M)); samples through the "
                    "synchronous call",
        "ms_per_sample": t_cl * 1e3,
        "edges_per_s": edges / reps / t_cl,
        "mean_edges_per_sample": edges / reps,
        "ms_per_rank_count_sample": t_rank * 1e3,
        "ms_triangle_count": t_tri * 1e3,
        "triangles_one_sample": tri_big,
        "bias": {"network": "Holme-Kim, 5000 nodes, m = 10, triad probability 0.1 (seeded)",
                 "replicas": R, "ubcm_fit_residual": fit.residual,
                 "holme_kim": {"rich_club_density": {f"{a:g}": v for a, v in zip(alphas, density(hk_counts))},
                               "triangles": hk_triangles(mh, hs, hd, hn, dev), "edges": int(len(hs))},
                 **stats,
                 "reading": "[mean, sd] over the replicas; rich-club density = edges among the top alpha of nodes "
                            "by degree / pairs among them"},
    }


def hk_triangles(mh, s, d, n, dev) -> int:
    import torch

    return mh.count_triangles(torch.as_tensor(s, device=dev), torch.as_tensor(d, device=dev), n)


def atomic_add_rate(dev, slots: int = 1 << 22, blocks: int = 2048, iters: int = 256) -> float:
    """Random int32 atomic adds per second on this GPU, from the probe library
    (libmh_probe.so): blocks x 256 lanes, each adding 1 to `iters` random
    counters of a table of `slots` (2^22 = 16 MB by default: the ensemble's
    degree arrays in use at one time are of that order).  The degree sink
    issues one such add per sampled edge, so this rate bounds it."""
    import torch

    import paper_2509_13230_amd as mh

    path = os.path.join(os.path.dirname(mh.__file__), "libmh_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2509_13230_amd.build`")
    P = ctypes.CDLL(path)
    P.mhp_atomic_adds.restype = ctypes.c_int
    P.mhp_atomic_adds.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    buf = torch.zeros(slots, dtype=torch.int32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    runs = []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = P.mhp_atomic_adds(ctypes.c_void_p(buf.data_ptr()), slots, blocks, iters, stream)
        torch.cuda.synchronize()
        if rc != 0:
            raise RuntimeError(f"mhp_atomic_adds failed ({rc})")
        if rep:
            runs.append(time.perf_counter() - t0)
    n_ops = blocks * 256 * iters
    assert int(buf.sum().item()) == 4 * n_ops
    return n_ops / min(runs)


def batched_ensemble(args, dev) -> dict:
    """The ensemble workload: 256 networks (N log-uniform in [1e3, 2e5],
    x = exp(Normal(-5, 2))) x 16 replicas = 4,096 samples, every network
    prepared once beforehand (timed separately).  Times the batched sampler
    writing edge lists (persistent launches over groups of samples whose edges
    fit one buffer) against the same 4,096 samples through the plain
    single-sample path (order + plan + sweep + edge output each), issued back
    to back through the asynchronous entry point (and, as a second figure,
    through the synchronous call, which reads each sample's edge count back);
    and the two degree-sink modes: one hipGraph launch adding degrees by
    atomics, and graphs over groups of samples counting columns through a slot
    buffer."""
    import torch

    import paper_2509_13230_amd as mh
    import workloads

    nets = workloads.cfg4_networks(seed=4, n_networks=args.batch_networks)
    xs = [torch.as_tensor(nw.x, device=dev) for nw in nets]
    R = args.batch_replicas
    net_ids = [i for i in range(len(xs)) for _ in range(R)]
    reps = [r for _ in xs for r in range(R)]
    S = len(net_ids)

    # batched: prepare once, autotune on a probe (seg_work and grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = mh.Batch(xs, seg_work=args.seg_work, max_samples=S)
    torch.cuda.synchronize()
    t_prepare = time.perf_counter() - t0
    probe = list(range(0, len(xs), max(1, len(xs) // 16)))
    tuned = b.autotune(probe, [0] * len(probe), seg_candidates=(8, 16, 32), grid_candidates=(0, 1024, 2048))
    sw = tuned["seg_work"]  # the plain samples use the same segment length

    # plain: every sample through the single-sample entry point
    max_n = max(x.numel() for x in xs)
    L = mh.lib()
    plan = mh.PlanParams(sw, 0, 0, 0, None)
    ws = torch.empty(L.mh_workspace_bytes(max_n, 0, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    # capacity: the largest sample seen on replica 0 of every network, with margin
    caps = []
    for x in xs:
        s_, _ = mh.sample_unweighted(x, seed=args.seed, replica=0, seg_work=sw, workspace=ws)
        caps.append(s_.numel())
    cap = int(max(caps) * 1.1) + 65536
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_counts = []
    for i, r in zip(net_ids, reps):
        s_, _ = mh.sample_unweighted(xs[i], seed=args.seed, replica=r, seg_work=sw, out=(src, dst),
                                     workspace=ws)
        plain_counts.append(s_.numel())
    plain_edges = sum(plain_counts)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # the same samples issued back to back through the asynchronous entry point
    # (no count readback between samples): the faster way to use the plain path
    for i, r in zip(net_ids[:8], reps[:8]):
        mh.sample_async(xs[i], None, (src, dst), ws, seed=args.seed, replica=r, seg_work=sw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in zip(net_ids, reps):
        mh.sample_async(xs[i], None, (src, dst), ws, seed=args.seed, replica=r, seg_work=sw)
    torch.cuda.synchronize()
    t_plain_async = time.perf_counter() - t0
    # the chains' steps (untimed, the statistics variant of the sweep): a
    # batched sample takes the same steps as its plain twin
    steps_total = 0
    for i, r in zip(net_ids, reps):
        _, _, st_ = mh.sample_unweighted(xs[i], seed=args.seed, replica=r, seg_work=sw, out=(src, dst),
                                         workspace=ws, stats=True)
        steps_total += st_["steps"]
    del src, dst, ws

    # batched: one graph launch per ensemble (prepared and tuned above)
    net_t = torch.tensor(net_ids, dtype=torch.int32, device=dev)
    rep_t = torch.tensor(reps, dtype=torch.int32, device=dev)
    off = b.degree_offsets(torch.tensor(net_ids))
    deg = torch.empty(int(off[-1]), dtype=torch.int32, device=dev)
    offd = off.to(dev)
    g = b.capture_degrees(net_t, rep_t, args.seed, deg, offd, grid_blocks=tuned["grid_blocks"])
    g.launch()  # warm-up
    b.result(-1)
    runs = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch()
        b.result(-1)
        runs.append(time.perf_counter() - t0)
    t_batch = min(runs)
    batch_edges = int(deg.sum().item()) // 2
    del g

    # the same degree sequences, columns counted through a slot buffer
    # (MH_BATCH_DEGREES_STAGED): samples in consecutive groups whose columns
    # fit the buffer with margin (a sample's region is sized from a bound on
    # its proposals; what overflows a region is added by atomics), one graph per
    # group, every group's degrees at its place in one array
    slot_cap = args.batch_slot_buffer
    sgroups, cur, need = [], [], 0
    for s_i, c in enumerate(plain_counts):
        w_ = (9 * c) // 5 + 4096
        if cur and need + w_ > slot_cap:
            sgroups.append(cur)
            cur, need = [], 0
        cur.append(s_i)
        need += w_
    sgroups.append(cur)
    slots = torch.empty(slot_cap, dtype=torch.int32, device=dev)
    sdeg = torch.empty_like(deg)
    graphs = []
    for grp in sgroups:
        gn = torch.tensor([net_ids[j] for j in grp], dtype=torch.int32, device=dev)
        gr = torch.tensor([reps[j] for j in grp], dtype=torch.int32, device=dev)
        goff = b.degree_offsets(gn.cpu())
        base = int(off[grp[0]])
        graphs.append(b.capture_degrees(gn, gr, args.seed, sdeg[base:base + int(goff[-1])], goff.to(dev),
                                        grid_blocks=tuned["grid_blocks"], slots=slots))
    for g_ in graphs:  # warm-up
        g_.launch()
    b.result(-1)
    runs = []
    for _ in range(2):
        sdeg.fill_(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g_ in graphs:
            g_.launch()
        b.result(-1)
        runs.append(time.perf_counter() - t0)
    t_staged = min(runs)
    staged_equal = bool(torch.equal(sdeg, deg))
    del deg, sdeg, slots, graphs

    # batched, edge output: the samples in consecutive groups whose edges fit
    # one output buffer (src, dst and the sample index, int32 each), one
    # persistent launch per group, the buffer reused like the plain samples'
    group_cap = args.batch_edge_buffer
    # room beyond a group's edges for the waves' output chunks (MH_BATCH_EDGE_SLACK)
    group_edges = group_cap - mh.BATCH_EDGE_SLACK
    groups, cur, cur_edges = [], [], 0
    for s_i, c in enumerate(plain_counts):
        if cur and cur_edges + c > group_edges:
            groups.append(cur)
            cur, cur_edges = [], 0
        cur.append(s_i)
        cur_edges += c
    groups.append(cur)
    esrc = torch.empty(group_cap, dtype=torch.int32, device=dev)
    edst = torch.empty(group_cap, dtype=torch.int32, device=dev)
    esid = torch.empty(group_cap, dtype=torch.int32, device=dev)
    gnet = [torch.tensor([net_ids[j] for j in grp], dtype=torch.int32, device=dev) for grp in groups]
    grep = [torch.tensor([reps[j] for j in grp], dtype=torch.int32, device=dev) for grp in groups]
    b.sample_edges_async(gnet[0], grep[0], args.seed, esrc, edst, None, esid, group_cap, tuned["grid_blocks"])
    b.result(group_cap)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edge_total = 0
    for gn, gr in zip(gnet, grep):
        b.sample_edges_async(gn, gr, args.seed, esrc, edst, None, esid, group_cap, tuned["grid_blocks"])
        m = b.result(group_cap)
        if m < 0:
            raise RuntimeError(f"batched edge output overflowed its buffer ({-m} edges)")
        edge_total += m
    torch.cuda.synchronize()
    t_batch_edges = time.perf_counter() - t0
    del esrc, edst, esid
    # The degree sink adds 1 to a column's counter per sampled edge (and each
    # row's count once per row): bound by the GPU's rate of random atomic adds.
    ceiling = atomic_add_rate(dev)

    def valu(t):
        ops = steps_total * SWEEP_VALU_PER_STEP / t
        return {"bound": "alu", "achieved": ops / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                "frac": ops / PEAK_LANE_OPS,
                "work": f"{steps_total} steps x {SWEEP_VALU_PER_STEP} VALU lane-ops over the whole call"}

    return {
        "workload": f"{len(xs)} networks x {R} replicas = {S} samples, N log-uniform in [1e3, 2e5], "
                    "x = exp(Normal(-5, 2)), unweighted",
        "samples": S,
        "edges": batch_edges,
        "plain_edges": plain_edges,
        # the same (network, replica, seed, seg_work) draws the same samples either way
        "plain_edges_equal": plain_edges == batch_edges,
        # like for like: both write every edge to HBM
        "replicas_per_s_batched": S / t_batch_edges,
        "replicas_per_s_plain": S / t_plain_async,
        "speedup_vs_plain": t_plain_async / t_batch_edges,
        "output": "edge lists (plain: src, dst; batched: src, dst and the sample index, in "
                  f"{len(groups)} launches of up to {group_edges} edges)",
        "batched_edges_equal": edge_total == plain_edges,
        "edges_per_s_batched": edge_total / t_batch_edges,
        "valu_batched": valu(t_batch_edges),
        "ms_batched_edges_total": t_batch_edges * 1e3,
        "replicas_per_s_plain_sync": S / t_plain,
        "ms_prepare": t_prepare * 1e3,
        "ms_plain_total": t_plain_async * 1e3,
        "ms_plain_sync_total": t_plain * 1e3,
        "replicas_per_s_batched_incl_prepare": S / (t_batch_edges + t_prepare),
        # a different output: per-sample degree sequences, no edge list
        "degree_sink": {"replicas_per_s": S / t_batch, "ms_graph_launch": t_batch * 1e3, "valu": valu(t_batch),
                        "edges_per_s": batch_edges / t_batch,
                        "speedup_vs_plain_edge_output": t_plain_async / t_batch,
                        # no published figure exists for this rate: the ceiling is measured
                        "atomic_ceiling": {"bound": "atomic", "achieved": batch_edges / t_batch, "ceiling": ceiling,
                                           "unit": "int32 atomic adds/s", "frac": batch_edges / t_batch / ceiling,
                                           "work_per_launch": f"{batch_edges} column adds (one per edge; per-row "
                                                              "adds not counted)",
                                           "ceiling_source": "measured here (libmh_probe.so): 2048 x 256 lanes x "
                                                             "256 random int32 atomic adds into 2^22 counters"}},
        # the same sequences through the slot buffer: the sweep writes each
        # accepted column (4 B), a counting kernel reads it per 32768-column window
        "degree_sink_staged": {"replicas_per_s": S / t_staged,
                               "ms_graph_launches": t_staged * 1e3, "edges_per_s": batch_edges / t_staged,
                               "launches": len(sgroups), "slot_buffer_int32": slot_cap,
                               "degrees_equal_atomic_sink": staged_equal,
                               "speedup_vs_atomic_sink": t_batch / t_staged,
                               "speedup_vs_plain_edge_output": t_plain_async / t_staged,
                               "valu": valu(t_staged)},
        "tuned": tuned,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seg-work", type=int, default=8)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--grid-blocks", type=int, default=0, help="sweep grid (0 = all resident blocks)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--bf-prefix", type=int, default=50_000,
                    help="nodes of the brute-force comparison network (0: skip it)")
    ap.add_argument("--deg-n", type=int, default=200_000,
                    help="nodes of the expected-degree measurement (0: skip it)")
    ap.add_argument("--w-n", type=int, default=200_000, help="nodes of the weighted measurement (0: skip it)")
    ap.add_argument("--w-fit-newton", type=int, default=200,
                    help="Newton steps of the weighted fit for the fitted-parameter measurement (0: skip it)")
    ap.add_argument("--w-seg-work", type=int, default=32,
                    help="seg_work of the weighted measurement (the best of 8-128 on that workload)")
    ap.add_argument("--bip-rows", type=int, default=1_000_000,
                    help="rows of the bipartite measurement, with half as many columns (0: skip it)")
    ap.add_argument("--bip-seg-work", type=int, default=8, help="seg_work of the two-set measurement")
    ap.add_argument("--accuracy-replicas", type=int, default=64,
                    help="replicas of the degree-accuracy comparison of MH and brute force")
    ap.add_argument("--bias-replicas", type=int, default=100,
                    help="replicas of the Chung-Lu bias statistics (0: skip the Chung-Lu measurement)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--batch-slot-buffer", type=int, default=4_000_000_000,
                    help="int32 slots of the staged degree sink's buffer")
    ap.add_argument("--skip-small", action="store_true", help="skip the N=2,000 timings")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy a buffer of this many MiB once first (reference for HBM byte counters)")
    ap.add_argument("--batch-networks", type=int, default=256)
    ap.add_argument("--batch-replicas", type=int, default=16)
    ap.add_argument("--batch-edge-buffer", type=int, default=1_500_000_000,
                    help="edges per launch of the batched edge-output measurement")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the sampler has no multi-GPU path (a sample's rows, or a "
              "batch's samples, would be split across GPUs with no communication between them).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_13230_amd as mh
    import workloads
    from paper_2509_13230_amd.fit import fit_ubcm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration_mib > 0:
        a = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev)
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy
    # the timed input: x fitted on the CPU to the power-law targets (stored,
    # one value per degree class); the device fit of the same targets runs
    # beside it (untimed) and is reported against it
    k_target = workloads.cfg2_degrees(seed=2, n=args.n)
    x_np = workloads.cfg2_fitted_x() if args.n == 1_000_000 else None
    t0 = time.perf_counter()
    fit = fit_ubcm(k_target, tol=1e-10)
    t_fit = time.perf_counter() - t0
    if x_np is None:
        x_np = fit.x
    fit_info = {"device_fit_iterations": fit.iterations, "device_fit_residual": fit.residual,
                "device_fit_s": t_fit,
                "device_fit_max_rel_diff_from_input": float(np.max(np.abs(fit.x - x_np) / x_np))}
    x = torch.as_tensor(x_np, device=dev)
    n = x.numel()
    print(f"# device fit: {fit.iterations} iterations, residual {fit.residual:.2e}, {t_fit:.2f} s", file=sys.stderr,
          flush=True)

    L = mh.lib()
    plan = mh.PlanParams(args.seg_work, 0, 0, 0, None)
    ws = torch.empty(L.mh_workspace_bytes(n, 0, ctypes.byref(plan)), dtype=torch.uint8, device=dev)
    s0, d0, st0 = mh.sample_unweighted(x, seed=args.seed, replica=0, seg_work=args.seg_work, stats=True,
                                       workspace=ws)
    cap = int(len(s0) * 1.05) + 65536
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    # Every fifth timed sample records 2 events, around the sweep (the kernel
    # the roofline is taken on): an event record leaves a ~4.5 us gap on the
    # stream even without the system fence, so the other samples record none.
    # The order and plan stages are timed on the untimed repeat below.
    timed_sweeps = [i for i in range(args.steps) if i % 5 == 0]
    ev = HipEvents(4 * args.steps, present=lambda i: (i // 4) % 5 == 0 and i % 4 >= 2)
    ev_size = ctypes.sizeof(ctypes.c_void_p)
    ev_stage = HipEvents(4 * args.steps)

    def step(replica, events=None):
        mh.sample_async(x, None, (src, dst), ws, seed=args.seed, replica=replica, seg_work=args.seg_work,
                        stage_events=events, grid_blocks=args.grid_blocks)

    for w in range(args.warmup):
        step(1 + w)
    torch.cuda.synchronize()
    replicas = [1000 + i for i in range(args.steps)]
    t0 = time.perf_counter()
    for i, r in enumerate(replicas):
        step(r, ev.address + 4 * i * ev_size)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last_edges = mh.sample_result(ws, cap)
    sweep_ms = sum(ev.elapsed_ms(4 * i + 2, 4 * i + 3) for i in timed_sweeps) / len(timed_sweeps)
    ms_per_step = elapsed / args.steps * 1e3

    # edges and algorithmic work of the timed samples (the same samples again,
    # untimed), and the stage times of the order and plan steps
    steps_total = 0
    steps_timed_sweeps = 0
    edges_timed_sweeps = 0
    edges = 0
    stage = np.zeros(3)
    for i, r in enumerate(replicas):
        _, _, st = mh.sample_unweighted(x, seed=args.seed, replica=r, seg_work=args.seg_work, stats=True,
                                        out=(src, dst), workspace=ws, grid_blocks=args.grid_blocks,
                                        stage_events=ev_stage.address + 4 * i * ev_size)
        stage += [ev_stage.elapsed_ms(4 * i, 4 * i + 1), ev_stage.elapsed_ms(4 * i + 1, 4 * i + 2),
                  ev_stage.elapsed_ms(4 * i + 2, 4 * i + 3)]
        steps_total += st["steps"]
        if i in timed_sweeps:
            steps_timed_sweeps += st["steps"]
            edges_timed_sweeps += st["n_edges"]
        edges += st["n_edges"]
    if st["n_edges"] != last_edges:
        raise RuntimeError(f"timed and repeated sample differ: {last_edges} vs {st['n_edges']} edges")
    value = edges / elapsed
    steps_per_sweep = steps_timed_sweeps / len(timed_sweeps)
    achieved_lane_ops = steps_per_sweep * SWEEP_VALU_PER_STEP / (sweep_ms * 1e-3)
    # the sweep's edge output against HBM bandwidth (8 B per edge written)
    edges_per_sweep = edges_timed_sweeps / len(timed_sweeps)
    write_gbs = edges_per_sweep * 8 / (sweep_ms * 1e-3) / 1e9
    # algorithmic bytes of one sweep launch: every node record (16 B) read once,
    # every edge (8 B) written once
    alg_bytes = 16 * n + edges_per_sweep * 8
    traffic = None
    if (sweep_sources_sha256() == SWEEP_COUNTERS["sources_sha256"]
            and workloads.sha256(x_np) == SWEEP_COUNTERS["input_sha256"]
            and args.seg_work == SWEEP_COUNTERS["seg_work"]):
        traffic = (SWEEP_COUNTERS["fetch_kib"] * 1024 * SWEEP_COUNTERS["fetch_scale"]
                   + SWEEP_COUNTERS["write_kib"] * 1024 * SWEEP_COUNTERS["write_scale"])
    roof = {"bound": "alu", "kernel": "k_sweep (unweighted)",
            "achieved": achieved_lane_ops / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
            "frac": achieved_lane_ops / PEAK_LANE_OPS, "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes": alg_bytes,
            "traffic_over_algorithmic": traffic / alg_bytes if traffic is not None else None,
            "work_per_launch": f"{steps_per_sweep:.0f} steps x {SWEEP_VALU_PER_STEP} VALU lane-ops",
            "timed_launches": len(timed_sweeps),
            "avg_launch_ms": sweep_ms,
            "hbm_write": {"achieved": write_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": write_gbs / HBM_PEAK_GBS, "bytes_per_launch": edges_per_sweep * 8}}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "UBCM, N=1,000,000, power-law target degrees (exponent 2.1, k in [1, 10^4]), "
                               "x fitted (class-compressed fixed point, residual 1e-10, stored CPU fit), one "
                               "sample per step, samples issued back to back on one stream",
                   "n": n, "seg_work": args.seg_work, "mean_edges_per_sample": edges / args.steps,
                   "input_sha256": workloads.sha256(x_np)},
        "fit": fit_info,
        "stages_ms": {"order": stage[0] / args.steps, "bound_plan": stage[1] / args.steps, "sweep": sweep_ms},
        "sweep_steps_per_sample": steps_total / args.steps,
        "sweep_only_edges_per_s": edges_per_sweep / (sweep_ms * 1e-3),
        "roofline": roof,
    }
    if not args.skip_small:
        out["small"] = small_bench(args, dev)
    if not args.skip_batched:
        out["batched"] = batched_ensemble(args, dev)
    if args.bf_prefix > 0:
        out["bruteforce"] = bruteforce_vs_mh(args, x, dev)
    if args.w_n > 0:
        out["weighted"] = weighted_bench(args, dev)
        if args.w_fit_newton > 0:
            out["weighted_fitted"] = weighted_bench(args, dev, fitted=True)
    if args.bip_rows > 0:
        out["bipartite"] = bipartite_bench(args, dev)
    if args.bias_replicas > 0:
        out["chung_lu"] = chung_lu_bench(args, dev)
    if args.deg_n > 0:
        out["expected_degree"] = expected_degree_bench(args, dev)
    if not args.no_cpu_baseline:
        def gpu_sample(replica):
            s_, d_ = mh.sample_unweighted(x, seed=args.seed, replica=replica, seg_work=args.seg_work,
                                          out=(src, dst), workspace=ws, grid_blocks=args.grid_blocks)
            return s_.cpu().numpy(), d_.cpu().numpy()

        # the timed samples' (seed, replica) pairs first, then further replicas
        out["cpu_baseline"] = cpu_baseline(x_np, args.seed, args.seg_work, args.cpu_budget,
                                           replicas + [1000 + args.steps + i for i in range(500)], gpu_sample)
        out["parity"] = out["cpu_baseline"]["parity"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
