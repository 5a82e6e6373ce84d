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
                       kernel="k_count_lin<PLANE3D>", compact="k_compact_lin<PLANE3D>", bound="hbm"),
    "pose4dof_1m": dict(desc="gravity-aligned 4-DoF pose: 1e6 matches in a 200 m box, 0.5% inliers with 0.5 deg "
                             "bearing noise, eps 0.5 m / 0.5 deg", kernel="k_count_pose<POSE4DOF>",
                        compact="k_compact<POSE4DOF>", bound="alu"),
    "ray3d_100k": dict(desc="ray intersection: 1e5 rays, 1% through a common centre", kernel="k_count_lin<RAY3D>",
                       compact="k_compact_lin<RAY3D>", bound="hbm"),
    "line2d_10k": dict(desc="2D line fitting by duality: 1e4 points, 5% inliers", kernel="k_count_lin<LINE2D>",
                       compact="k_compact_lin<LINE2D>", bound="hbm"),
    "pose4dof_serve256": dict(desc="256 independent 4-DoF pose problems, matches log-uniform in [1e3, 2e5], inlier "
                                   "ratio log-uniform in [0.2%, 10%], served through gv_submit/gv_poll",
                              kernel="k_count_pose<POSE4DOF>", bound="alu"),
}


def serve_bench(args):
    """Plain binary64, one problem at a time (gv_solve) against the binary32
    filter with continuous batching (gv_submit/gv_poll, three lanes), same 256
    problems, inputs resident in HBM; then Poisson arrivals for p50/p99
    latency, beside the plain form's FIFO latency on the same arrivals."""
    import threading
    import numpy as np
    from paper_2107_11810_amd import gvote, synth
    probs = synth.batch_pose4dof(n_problems=256)
    print(f"{len(probs)} problems, {sum(len(g['cols'][0]) for g in probs)} matches", file=sys.stderr, flush=True)
    ctx = gvote.Context(0)
    cols = [gvote.to_device(g["cols"]) for g in probs]
    hip = gvote.hip()
    g0 = probs[0]
    ctx.solve(g0["family"], cols[0], g0["lo"], g0["hi"], g0["eps"])  # warm-up
    hip.hipDeviceSynchronize()
    plain, dur = [], []
    t0 = time.perf_counter()
    for g, c in zip(probs, cols):
        t1 = time.perf_counter()
        plain.append(ctx.solve(g["family"], c, g["lo"], g["hi"], g["eps"], precision=gvote.FP64_PLAIN))
        dur.append(time.perf_counter() - t1)
    t_plain = time.perf_counter() - t0
    print(f"plain binary64 one at a time: {t_plain:.2f} s", file=sys.stderr, flush=True)
    slow = sorted(range(len(dur)), key=lambda i: -dur[i])[:5]
    print("slowest plain solves: " + ", ".join(
        f"#{i} n={len(probs[i]['cols'][0])} {dur[i]*1e3:.0f} ms (library {plain[i]['stats']['ms_total']:.0f} ms, "
        f"{plain[i]['stats']['tests']:.3g} tests)" for i in slow), file=sys.stderr, flush=True)

    def submit_all(order_times=None, tickets=None, arrivals=None):
        tickets = [] if tickets is None else tickets
        arrivals = [] if arrivals is None else arrivals
        t_start = time.perf_counter()
        for i, (g, c) in enumerate(zip(probs, cols)):
            if order_times is not None:
                dt = order_times[i] - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
            # the arrival time is recorded before the ticket becomes visible
            arrivals.append(time.perf_counter())
            tickets.append(gvote.submit(ctx, g["family"], c, g["lo"], g["hi"], g["eps"], precision=args.precision))
        return tickets, arrivals

    def collect(tickets, box, n_total):
        """Poll every ticket as soon as it exists (tickets may still be
        arriving from another thread); completion time = first successful
        poll, polled every 0.2 ms."""
        done = [None] * n_total
        res = [None] * n_total
        left = set(range(n_total))
        while left:
            avail = len(tickets)
            for i in list(left):
                if i >= avail:
                    continue
                st, r = gvote.poll(ctx, tickets[i], len(probs[i]["cols"][0]), timeout_ms=0)
                if st == 0:
                    done[i] = time.perf_counter()
                    res[i] = r
                    left.discard(i)
                elif st != -5:
                    raise RuntimeError(f"poll failed: {st}")
            time.sleep(0.0002)
        box.extend([done, res])

    t0 = time.perf_counter()
    tk, _ = submit_all()
    box = []
    collect(tk, box, len(probs))
    t_batch = time.perf_counter() - t0
    same = all(r["count"] == p["count"] and r["leaf_index"] == p["leaf_index"] for r, p in zip(box[1], plain))
    mu = len(probs) / t_batch
    print(f"filter + continuous batching: {t_batch:.2f} s, identical={same}", file=sys.stderr, flush=True)
    lat, fifo = {}, {}
    for frac in (0.8, 0.5):
        arr = synth.poisson_arrivals(len(probs), frac * mu, seed=199)
        tickets, arrivals = [], []

        def sub():
            submit_all(arr, tickets, arrivals)
        th = threading.Thread(target=sub)
        th.start()
        box2 = []
        collect(tickets, box2, len(probs))
        th.join()
        L = np.array(box2[0]) - np.array(arrivals)
        lat[frac] = (float(np.percentile(L, 50)), float(np.percentile(L, 99)))
        # the plain form on the same arrival times: one solve at a time in
        # arrival order, each taking its measured binary64 duration
        fin, done_t = [], 0.0
        for a, d in zip(arr, dur):
            done_t = max(done_t, a) + d
            fin.append(done_t - a)
        fifo[frac] = (float(np.percentile(fin, 50)), float(np.percentile(fin, 99)))
        print(f"arrivals at {frac:.1f} x saturated rate: p50 {lat[frac][0]*1e3:.1f} ms, p99 {lat[frac][1]*1e3:.1f} ms"
              f" (plain FIFO on the same arrivals: p50 {fifo[frac][0]*1e3:.1f} ms, p99 {fifo[frac][1]*1e3:.1f} ms)",
              file=sys.stderr, flush=True)
    ctx.close()
    out = {
        "metric": "solves/s", "value": mu, "unit": "solves/s", "n_gpus": 1, "steps": len(probs), "warmup": 1,
        "ms_per_step": 1e3 * t_batch / len(probs), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "pose4dof_serve256", "description": WORKLOADS["pose4dof_serve256"]["desc"],
                   "n_problems": len(probs), "total_matches": int(sum(len(g["cols"][0]) for g in probs))},
        "plain_fp64_solves_per_s": len(probs) / t_plain,
        "batched_over_plain": (len(probs) / t_plain and mu / (len(probs) / t_plain)),
        "identical_to_plain": same,
        "latency_ms": {f"{f}x_saturated": {"p50": lat[f][0] * 1e3, "p99": lat[f][1] * 1e3} for f in lat},
        "plain_fifo_latency_ms": {f"{f}x_saturated": {"p50": fifo[f][0] * 1e3, "p99": fifo[f][1] * 1e3} for f in fifo},
    }
    print(json.dumps(out), flush=True)



def calibrate_copy(nbytes=1 << 30, reps=3):
    """Device-to-device copies of a known size: the scale for the memory
    counters (bytes a counter reports per byte a plain copy must move)."""
    import ctypes
    from paper_2107_11810_amd import gvote
    hip = gvote.hip()
    src, dst = ctypes.c_void_p(), ctypes.c_void_p()
    if hip.hipMalloc(ctypes.byref(src), nbytes) or hip.hipMalloc(ctypes.byref(dst), nbytes):
        raise RuntimeError("hipMalloc failed")
    for _ in range(reps):
        if hip.hipMemcpy(dst, src, nbytes, 3):  # device -> device
            raise RuntimeError("hipMemcpy failed")
    hip.hipDeviceSynchronize()
    hip.hipFree(src)
    hip.hipFree(dst)
    print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": reps}), flush=True)


def per_kernel(name, ms, nbytes, launches, steps):
    """Achieved algorithmic HBM rate of one kernel over the timed solves."""
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"kernel": name, "launches": launches, "ms_per_step": round(ms / steps, 2),
            "bytes_per_launch": int(nbytes / launches) if launches else None,
            "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the kernel from the committed memory-counter
    record (profiles/traffic.json), or None when there is none or the kernel
    sources changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[workload]
    except (OSError, KeyError, ValueError):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2107_11810_amd", "csrc", f), "rb").read()
                   for f in ("gv_device.h", "gv_kernels.h"))
    if rec.get("kernel") != kernel or rec.get("sources_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return int(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def measured_valu(workload, kernel):
    """VALU lane-operations per incidence test of the kernel from the
    committed counter record (profiles/valu.json), or None when there is
    none or the kernel sources changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "valu.json")))[workload]
    except (OSError, KeyError, ValueError):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2107_11810_amd", "csrc", f), "rb").read()
                   for f in ("gv_device.h", "gv_kernels.h"))
    if rec.get("sources_sha256") != hashlib.sha256(src).hexdigest():
        return None
    per_kernel_ops = rec.get("kernels", {rec.get("kernel"): rec.get("lane_ops_per_test")})
    v = per_kernel_ops.get(kernel)
    return float(v) if v is not None else None


def valu_frac(opt, tests, ms):
    """Fraction of the non-packed VALU peak that opt lane-operations per test
    over the given tests take in ms of kernel time."""
    return round(opt * tests / (ms * 1e-3) / VALU_LANE_OPS, 4) if ms > 0 else None


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
    ap.add_argument("--warmup", type=int, default=3, help="untimed solves first (they include the autotuning)")
    ap.add_argument("--workload", default="plane3d_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-tests", type=float, default=2.5e8, help="oracle sample size (incidence tests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=1, help="0 binary64, 1 binary32 filter")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 1 GiB device copies (scale for the memory counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    if args.workload == "pose4dof_serve256":
        serve_bench(args)
        return
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
        kname, kms, kb, kn = W["compact"], c_ms, c_b, c_n
    achieved = (kb / kn) / (kms / kn * 1e-3) / 1e9 if kn and kms > 0 else 0.0
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, kname),
            "launches": kn, "avg_launch_us": round(kms / kn * 1e3, 2) if kn else None,
            "bytes_per_launch": int(kb / kn) if kn else None,
            "kernel_ms_per_step": round(kms / len(results), 2),
            "other_kernel_ms_per_step": round((c_ms if kname == W["kernel"] else t_ms) / len(results), 2),
            # both big kernels: the incidence test (count pass) and compaction
            "kernels": [per_kernel(W["kernel"], t_ms, t_b, t_n, len(results)),
                        per_kernel(W["compact"], c_ms, c_b, c_n, len(results))]}
    # measured vector-ALU issue of each kernel beside its HBM figure
    for k, ms in zip(roof["kernels"], (t_ms, c_ms)):
        opt_k = measured_valu(args.workload, k["kernel"])
        if opt_k is not None:
            k["valu_frac"] = valu_frac(opt_k, tests, ms)
    if W["bound"] == "alu" and kname == W["kernel"]:
        # the incidence kernel of this family is bound by vector ALU work:
        # lane-operations per test (counted once with rocprofv3, see
        # profiles/valu.json) times the tests, over its event time
        opt = measured_valu(args.workload, kname)
        if opt is not None and kms > 0:
            ach = opt * tests / (kms * 1e-3) / 1e12
            roof.update({"bound": "alu", "achieved": round(ach, 2), "peak": VALU_LANE_OPS / 1e12,
                         "unit": "T lane-ops/s", "frac": round(ach / (VALU_LANE_OPS / 1e12), 4),
                         "lane_ops_per_test": round(opt, 2)})
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
