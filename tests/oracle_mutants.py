"""Planted mistakes in the oracle, and the pins that must catch them.

Each entry of MUTANTS names one plausible mistake (a dropped term, a wrong
sign, index, word or bound, a missing update), the text of mh_oracle.c it
replaces, and the pins (test functions of the oracle's CPU suite) expected to
fail once it is planted.  test_oracle_mutations.py builds every altered copy
with gcc and runs its pins in a child process (this file, run as a script):

    python tests/oracle_mutants.py <liboracle variant> <mutant name>

prints one JSON line {pin: "pass" | "fail: ..."}.  A mutant survives if all
of its pins pass.  The same pins must pass on the unaltered source.
"""
from __future__ import annotations

import json
import os
import sys
import traceback

# (name, old text, new text, occurrence to replace (0-based), pins)
# a pin is (module, function, keyword arguments)
MUTANTS = [
    ("uecm accept drops the -b of the denominator",
     "lhs = (U2 * tq) * (e + t);", "lhs = (U2 * tq) * (1.0 + t);", 0,
     [("test_oracle_sampler", "test_uecm_joint_law_and_weights", {"seg_work": 0})]),
    ("skip with the wrong sign",
     "return -log(u1) / log1p(tq / c);", "return log(u1) / log1p(tq / c);", 0,
     [("test_oracle_sampler", "test_skip_law_chi2", {"tq": 1.0, "c": 1.0}),
      ("test_oracle_sampler", "test_skip_endpoints_and_monotone", {})]),
    ("skip through log(1 + t) instead of log1p",
     "return -log(u1) / log1p(tq / c);", "return -log(u1) / log(1.0 + tq / c);", 0,
     [("test_oracle_sampler", "test_skip_mean_at_tiny_q", {"q": 1e-18, "c": 1.0})]),
    ("skip from 1 - q after q is rounded",
     "return -log(u1) / log1p(tq / c);", "return log(u1) / log(1.0 - tq / (c + tq));", 0,
     [("test_oracle_sampler", "test_skip_mean_at_tiny_q", {"q": 1e-18, "c": 1.0})]),
    ("proposal probability never updated",
     "                tq = t;\n                pos = j;", "                pos = j;", 0,
     [("test_oracle_sampler", "test_proposal_count_matches_exact_law", {})]),
    ("candidate probability read at the previous column",
     "double t = s * zs[j];", "double t = s * zs[pos];", 0,
     [("test_oracle_sampler", "test_ubcm_joint_law_chi2", {"seg_work": 0})]),
    ("bound over the unprocessed nodes without the focal node",
     "        if (v > y1) { y2 = y1; y1 = v; }\n        else if (v > y2) { y2 = v; }\n"
     "        double Y = (y2 < 0.0) ? 0.0 : y1 * y2;\n        c[r] = 1.0 - Y;\n",
     "        double Y = (y2 < 0.0) ? 0.0 : y1 * y2;\n        c[r] = 1.0 - Y;\n"
     "        if (v > y1) { y2 = y1; y1 = v; }\n        else if (v > y2) { y2 = v; }\n", 0,
     [("test_oracle_sampler", "test_bound_brute_force", {})]),
    ("acceptance uniform taken from the skip's words",
     "double U2 = mho_u53(u[2], u[3]);", "double U2 = mho_u53(u[0], u[1]);", 0,
     [("test_oracle_sampler", "test_ubcm_joint_law_chi2", {"seg_work": 0})]),
    ("weight one too small",
     "return 1 + (int32_t)ratio;", "return (int32_t)ratio;", 0,
     [("test_oracle_sampler", "test_uecm_joint_law_and_weights", {"seg_work": 0}),
      ("test_oracle_sampler", "test_weighted_bf_joint_law_and_weights", {})]),
    ("weight law with b and 1 - b swapped",
     "double ratio = log(u) / log(b);", "double ratio = log(u) / log(1.0 - b);", 0,
     [("test_oracle_sampler", "test_uecm_joint_law_and_weights", {"seg_work": 0}),
      ("test_oracle_sampler", "test_weighted_bf_joint_law_and_weights", {})]),
    ("weighted brute force draws the weight from the existence uniform",
     "wt = draw_weight(mho_u53(u[2], u[3]), y[i] * y[j], &sat, &tie);",
     "wt = draw_weight(mho_u53(u[0], u[1]), y[i] * y[j], &sat, &tie);", 0,
     [("test_oracle_sampler", "test_weighted_bf_joint_law_and_weights", {})]),
    ("weighted brute force existence without the -b term",
     "double e = y ? 1.0 - y[i] * y[j] : 1.0;", "double e = 1.0;", 0,
     [("test_oracle_sampler", "test_weighted_bf_joint_law_and_weights", {})]),
    ("expected strength divides by 1 + b",
     "*e = *p / (1.0 - b);", "*e = *p / (1.0 + b);", 0,
     [("test_oracle_degree", "test_two_block_closed_form_weighted", {})]),
    ("wrong derivative of p with respect to b",
     "double dpb = a / D2;", "double dpb = b / D2;", 0,
     [("test_oracle_degree", "test_gradient_central_differences", {"weighted": True})]),
    ("order ties by descending id",
     "return (a > b) - (a < b);", "return (a < b) - (a > b);", 0,
     [("test_oracle_sampler", "test_order_matches_lexsort", {})]),
    ("uniform on [0, 1) instead of (0, 1]",
     "return (double)(m + 1u) * 0x1.0p-53;", "return (double)(m) * 0x1.0p-53;", 0,
     [("test_oracle_rng", "test_u53_range_endpoints", {})]),
    ("Philox key schedule with one Weyl constant twice",
     "k1 += PHILOX_W1;", "k1 += PHILOX_W0;", 0,
     [("test_oracle_rng", "test_philox_known_answers", None)]),
    ("plan rounds the dense segments down",
     "rp.nd = (rp.J - r - 1 + T - 1) / T;", "rp.nd = (rp.J - r - 1) / T;", 0,
     [("test_oracle_sampler", "test_plan_partitions_rows", {"seg_work": 3})]),
    ("directed sampler keeps self-loops",
     "if (lhs < rhs && !(exclude_self && id_j == id_r)) {", "if (lhs < rhs) {", 0,
     [("test_oracle_bipartite", "test_directed_joint_law_no_self_loops", {"weighted": False})]),
    ("bipartite bound from the smallest column y",
     "if (yr && yc[j] > ymax_c) ymax_c = yc[j];", "if (yr && (ymax_c == 0.0 || yc[j] < ymax_c)) ymax_c = yc[j];", 0,
     [("test_oracle_bipartite", "test_bipartite_weighted_joint_law_and_weights", {"seg_work": 0})]),
    ("Chung-Lu proposal not capped at 1",
     "lhs = U2 * (tq < 1.0 ? tq : 1.0);", "lhs = U2 * tq;", 0,
     [("test_oracle_chung_lu", "test_chung_lu_joint_law_chi2", {"seg_work": 0})]),
    ("Chung-Lu skip with the unweighted model's log(1 - q)",
     "return -log(u1) / -log1p(-tq);", "return -log(u1) / log1p(tq);", 0,
     [("test_oracle_chung_lu", "test_chung_lu_joint_law_chi2", {"seg_work": 0}),
      ("test_oracle_chung_lu", "test_homogeneous_chung_lu_is_erdos_renyi", {})]),
    ("triangle counted at every common neighbour",
     "if (adj[i] > b) ++tri;", "++tri;", 0,
     [("test_oracle_chung_lu", "test_triangles_brute_force", {}),
      ("test_oracle_chung_lu", "test_triangles_closed_forms", {})]),
]


def mutate(src: str, old: str, new: str, occurrence: int) -> str:
    start = -1
    for _ in range(occurrence + 1):
        start = src.find(old, start + 1)
        if start < 0:
            raise ValueError(f"text to replace not found: {old!r}")
    return src[:start] + new + src[start + len(old):]


def _run_pin(module: str, func: str, kwargs):
    import importlib

    mod = importlib.import_module(module)
    f = getattr(mod, func)
    if kwargs is None:
        # every parameter set of a parametrized pin (read from its mark)
        for mark in getattr(f, "pytestmark", []):
            if mark.name == "parametrize":
                names = [s.strip() for s in mark.args[0].split(",")]
                for vals in mark.args[1]:
                    vals = vals if isinstance(vals, tuple) else (vals,)
                    f(**dict(zip(names, vals)))
                return
        f()
    else:
        f(**kwargs)


def main(lib_path: str, name: str) -> None:
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    sys.path.insert(0, os.path.dirname(here))
    import oracle

    oracle.use_library(lib_path)
    pins = next(m[4] for m in MUTANTS if m[0] == name) if name != "*" else \
        sorted({(p[0], p[1], json.dumps(p[2], sort_keys=True)) for m in MUTANTS for p in m[4]})
    if name == "*":
        pins = [(a, b, json.loads(c)) for a, b, c in pins]
    out = {}
    for module, func, kwargs in pins:
        key = f"{module}::{func}{'' if not kwargs else kwargs}"
        try:
            _run_pin(module, func, kwargs)
            out[key] = "pass"
        except Exception as e:  # noqa: BLE001 -- a failing pin is the result
            out[key] = "fail: " + (str(e).splitlines()[0][:120] if str(e) else type(e).__name__)
        except BaseException:  # pytest.fail / skip raise BaseException subclasses
            out[key] = "fail: " + traceback.format_exc().splitlines()[-1][:120]
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
