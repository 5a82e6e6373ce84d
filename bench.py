#!/usr/bin/env python3
"""Benchmark of the voting hot path on one MI355X.

One step = one full solve (front end, root canonization, dive, depth-first
expansion with pruning, best-key reduction, inlier replay) of the 3D
plane-fitting workload: n = 1,000,000 points in the unit cube, 1% planted
inliers on a random plane with vertical noise sigma = 0.001, eps = 0.003 on
every dual axis, inputs resident in HBM before the timed region.

Prints one JSON line with the incidence-test throughput of the whole job,
the roofline figure of the dominant kernel (HIP events on the solve stream,
inside the library) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_FP32_TFLOPS = 157.3
# binary32 VALU lane-ops: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed)
VALU_LANE_OPS = 256 * 64 * 2.4e9

WORKLOADS = {
    "plane3d_1m": dict(desc="3D plane fitting by point-plane duality: n=1e6 points in the unit cube, 1% inliers "
                            "on a random plane with vertical noise 0.001, eps 0.003 on (a1, a2, a0)",
                       kernel="k_count_lin<PLANE3D>", bound="hbm"),
    "pose4dof_1m": dict(desc="gravity-aligned 4-DoF pose: 1e6 matches in a 200 m box, 0.5% inliers with 0.5 deg "
                             "bearing noise, eps 0.5 m / 0.5 deg", kernel="k_count_pose<EntQ32>", bound="alu"),
    "ray3d_100k": dict(desc="ray intersection: 1e5 rays, 1% through a common centre", kernel="k_count_lin<RAY3D>",
                       bound="hbm"),
    "line2d_10k": dict(desc="2D line fitting by duality: 1e4 points, 5% inliers", kernel="k_count_lin<LINE2D>",
                       bound="hbm"),
}


def cpu_baseline(g, budget_tests):
    """The oracle as it stands, single thread, stopped after a fixed number
    of incidence tests of the same solve."""
    import oracle
    pr = oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], test_budget=int(budget_tests))
    r = oracle.solve(pr)
    return {"value": r["tests"] / r["seconds"], "unit": "tests/s", "cores": 1, "kind": "oracle",
            "sample": f"first {r['tests']:.3g} incidence tests of the same solve (greedy dive then depth-first "
                      f"search), one host thread, {r['seconds']:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plane3d_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-tests", type=float, default=2.5e8, help="oracle sample size (incidence tests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=1, help="0 binary64, 1 binary32 filter")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    from paper_2107_11810_amd import gvote, synth
    W = WORKLOADS[args.workload]
    g = synth.config(args.workload)
    n = len(g["cols"][0])
    ctx = gvote.Context(0, kernel_timing=True)
    cols = gvote.to_device(g["cols"])  # inputs resident in HBM
    hip = gvote.hip()

    def solve():
        return ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], precision=args.precision)

    for i in range(args.warmup):
        r = solve()
        print(f"warmup {i}: count={r['count']} tests={r['stats']['tests']:.3g} "
              f"{r['stats']['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    hip.hipDeviceSynchronize()
    results = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(solve())
    hip.hipDeviceSynchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    for i, r in enumerate(results):
        print(f"step {i}: count={r['count']} inliers={r['n_inliers']} tests={r['stats']['tests']:.3g} "
              f"{r['stats']['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    counts = {(r["count"], r["leaf_index"]) for r in results}
    tests = sum(r["stats"]["tests"] for r in results)
    st = [r["stats"] for r in results]
    t_ms = sum(s["test_ms"] for s in st)
    c_ms = sum(s["compact_ms"] for s in st)
    t_b = sum(s["test_bytes"] for s in st)
    c_b = sum(s["compact_bytes"] for s in st)
    t_n = sum(s["test_launches"] for s in st)
    c_n = sum(s["compact_launches"] for s in st)
    if t_ms >= c_ms:
        kname, kms, kb, kn = W["kernel"], t_ms, t_b, t_n
    else:
        kname, kms, kb, kn = "k_compact", c_ms, c_b, c_n
    achieved = (kb / kn) / (kms / kn * 1e-3) / 1e9 if kn and kms > 0 else 0.0
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "launches": kn, "avg_launch_us": round(kms / kn * 1e3, 2) if kn else None,
            "bytes_per_launch": int(kb / kn) if kn else None,
            "kernel_ms_per_step": round(kms / len(results), 2),
            "other_kernel_ms_per_step": round((c_ms if kname != "k_compact" else t_ms) / len(results), 2)}
    out = {
        "metric": "incidence tests/s",
        "value": tests / sec,
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if g["family"] != "pose4dof" else ("f32+f64" if args.precision else "f64"),
        "data": "synthetic",
        "config": {"workload": args.workload, "description": W["desc"], "n": n, "eps": g["eps"],
                   "canon_c": 1.0, "precision": "fp32_filter" if args.precision else "fp64_plain"},
        "solves_per_s": args.steps / sec,
        "tests_per_solve": tests / args.steps,
        "count": results[0]["count"],
        "deterministic": len(counts) == 1,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_tests)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
