#!/usr/bin/env python3
"""Benchmark of the voting hot path on one MI355X.

One step = one full solve (front end, root canonization, dive, depth-first
expansion with pruning, best-key reduction, inlier replay) of the 3D
plane-fitting workload: n = 1,000,000 points in the unit cube, 1% planted
inliers on a random plane with vertical noise sigma = 0.001, eps = 0.003 on
every dual axis, inputs resident in HBM before the timed region.

Prints one JSON line: the incidence-test throughput of the whole job, the
roofline figure of the dominant kernel (HIP events on the solve stream,
inside the library), the CPU oracle timed on a bounded sample (one thread
and all cores), and, as extra keys, the 4-DoF pose workload (1e6 matches),
the 5-DoF pose workload with unknown focal length (2e4 matches), the
verification and refinement after the vote on both pose workloads, and the
256-problem serving workload (solves/s batched against plain, p50/p99
latency).  Every result is compared with the oracle's golden file
for its workload (tests/golden/); a mismatch exits non-zero.
"""
import argparse
import json
import math
import os
import sys
import time

# HIP gives a process four hardware queues unless told otherwise.  The
# serving lanes (three streams) and the context's own stream then share
# them, and a lane whose stream shares a queue waits behind the other's
# kernels; with eight queues every stream has its own.  Read once, when the
# process first initializes HIP, so it is set before anything else runs
# (raised to eight where the environment asks for fewer).
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
except ValueError:
    _hwq = 0
if _hwq < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def median(xs):
    v = sorted(xs)
    h = len(v) // 2
    return float(v[h]) if len(v) % 2 else 0.5 * (v[h - 1] + v[h])

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
    "pose5dof_20k": dict(desc="gravity-aligned pose with unknown focal length (x, y, z, yaw, f): 2e4 matches, 1.5% "
                              "inliers with 0.5 deg bearing noise, camera within 50 m / 5 m of the truth, f within "
                              "[0.6, 1.3] of it, eps 0.5 m / 0.5 deg / 1% of f", kernel="k_count_pose5<POSE5DOF>",
                         compact="k_compact<POSE5DOF>", bound="alu"),
    "ray3d_100k": dict(desc="ray intersection: 1e5 rays, 1% through a common centre", kernel="k_count_lin<RAY3D>",
                       compact="k_compact_lin<RAY3D>", bound="hbm"),
    "line2d_10k": dict(desc="2D line fitting by duality: 1e4 points, 5% inliers", kernel="k_count_lin<LINE2D>",
                       compact="k_compact_lin<LINE2D>", bound="hbm"),
    "sim2d_90k": dict(desc="similarity pointset alignment: 10,000 points, 9 candidate correspondences each (90,000 "
                           "surfaces), 1,000 true pairs under a planted similarity with noise 0.002, eps 0.01 on "
                           "(a, b, c, d)", kernel="k_count_lin<SIM2D>", compact="k_compact_lin<SIM2D>", bound="hbm"),
    "pose4dof_serve256": dict(desc="256 independent 4-DoF pose problems, matches log-uniform in [1e3, 2e5], inlier "
                                   "ratio log-uniform in [0.2%, 10%], served through gv_submit/gv_poll",
                              kernel="k_count_pose<POSE4DOF>", bound="alu"),
}


def _inl_sha(inl):
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(np.sort(inl), dtype="<i8").tobytes()).hexdigest()


def load_golden(workload):
    """The oracle's results for a workload (tests/golden/, written by a
    script that calls only the oracle), or None."""
    try:
        return json.load(open(os.path.join(ROOT, "tests", "golden", workload + ".json")))
    except (OSError, ValueError):
        return None


def golden_match(r, gold):
    k = len(gold["point"])  # axes of the family; the library reports 0 beyond them
    return (r["count"] == gold["count"] and r["leaf_index"] == gold["leaf_index"] and r["sector"] == gold["sector"]
            and r["n_inliers"] == gold["n_inliers"] and _inl_sha(r["inliers"]) == gold["inliers_sha256"]
            and [float(x) for x in r["point"][:k]] == gold["point"] and not any(r["point"][k:]))


def serve_bench(args, ctx=None):
    """Plain binary64, one problem at a time (gv_solve) against the binary32
    filter with continuous batching (gv_submit/gv_poll, three lanes), same 256
    problems, inputs resident in HBM; then Poisson arrivals for p50/p99
    latency, beside the plain form's FIFO latency on the same arrivals.
    Returns the figures and whether every result equals the oracle's."""
    import threading
    import numpy as np
    from paper_2107_11810_amd import gvote, synth
    probs = synth.batch_pose4dof(n_problems=256)
    print(f"{len(probs)} problems, {sum(len(g['cols'][0]) for g in probs)} matches", file=sys.stderr, flush=True)
    own = ctx is None
    ctx = gvote.Context(0) if own else ctx
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
    batched = box[1]
    same = all(r["count"] == p["count"] and r["leaf_index"] == p["leaf_index"] and r["sector"] == p["sector"]
               and np.array_equal(r["inliers"], p["inliers"]) for r, p in zip(batched, plain))
    mu = len(probs) / t_batch
    print(f"filter + continuous batching: {t_batch:.2f} s, identical={same}", file=sys.stderr, flush=True)
    lat, fifo, served = {}, {}, []
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
        served.append(box2[1])
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
    if own:
        ctx.close()
    gold = load_golden("pose4dof_serve256")
    golden = None
    if gold is not None and len(gold["problems"]) == len(probs):
        ok = all(golden_match(r, gg) for r, gg in zip(batched, gold["problems"]))
        ok = ok and all(golden_match(r, gg) for r, gg in zip(plain, gold["problems"]))
        ok = ok and all(golden_match(r, gg) for rs in served for r, gg in zip(rs, gold["problems"]))
        golden = {"problems": len(probs), "matches": ok,
                  "oracle_tests": int(sum(gg["oracle_tests"] for gg in gold["problems"])),
                  "gpu_tests_plain": int(sum(r["stats"]["tests"] for r in plain)),
                  "oracle_wall_s": round(sum(gg["oracle_wall_s"] for gg in gold["problems"]), 1),
                  "oracle_threads": gold.get("threads")}
    return {
        "solves_per_s": mu, "plain_fp64_solves_per_s": len(probs) / t_plain,
        "batched_over_plain": mu / (len(probs) / t_plain), "ms_batched": 1e3 * t_batch, "ms_plain": 1e3 * t_plain,
        "identical_to_plain": same,
        "latency_ms": {f"{f}x_saturated": {"p50": lat[f][0] * 1e3, "p99": lat[f][1] * 1e3} for f in lat},
        "plain_fifo_latency_ms": {f"{f}x_saturated": {"p50": fifo[f][0] * 1e3, "p99": fifo[f][1] * 1e3}
                                  for f in fifo},
        "n_problems": len(probs), "total_matches": int(sum(len(g["cols"][0]) for g in probs)),
        "golden": golden,
    }


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


def kernel_sources_sha256():
    """SHA-256 of every HIP source of the library (sorted by name): a counter
    record taken on other sources no longer describes the kernels."""
    import hashlib
    d = os.path.join(ROOT, "paper_2107_11810_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the kernel from the committed memory-counter
    record (profiles/traffic.json), or None when there is none or the kernel
    sources changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[workload]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    return int(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def measured_valu(workload, kernel):
    """VALU lane-operations per incidence test of the kernel from the
    committed counter record (profiles/valu.json), or None when there is
    none or the kernel sources changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "valu.json")))[workload]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    per_kernel_ops = rec.get("kernels", {rec.get("kernel"): rec.get("lane_ops_per_test")})
    v = per_kernel_ops.get(kernel)
    return float(v) if v is not None else None


def valu_frac(opt, tests, ms):
    """Fraction of the non-packed VALU peak that opt lane-operations per test
    over the given tests take in ms of kernel time."""
    return round(opt * tests / (ms * 1e-3) / VALU_LANE_OPS, 4) if ms > 0 else None


# Operations per incidence test of the 4-DoF predicate, counted from its
# definition (the binary64 surface/box test: the z half and the kappa cone
# half of the Sec. 4.2.1 surface), amortized over the 16 children of a cell
# that share an (x, y) part, a z bit or a kappa bit.  Per surface and cell:
#   z bits (2): 2 differences, the orientation by the sign of eta (1
#     compare, 2 negations, 3 selects), the squares a^2, T_lo^2, T_hi^2
#     (a^2 once): 21
#   kappa bits (2): the padded ends (2) and the two edge directions
#     (2 products, 4 sums): 16
#   (x, y) parts (4), 111 each: the rectangle (4), r_min^2 (4 compares,
#     4 selects, 2 products, 1 sum), r_max^2 (4 products, 2 max, 1 sum),
#     silhouette corners (4 compares, 12 selects), apex guard (1); per z
#     bit 2 products, 4 compares, 3 and/or (2 x 9); per kappa bit 4 cross
#     products (3 each), 8 sign compares, 7 and/or (2 x 27): 444
#   child masks: 16
# = 497 operations for 16 tests.  The binary32 filter's error bounds are not
# counted: they are the implementation's cost, not the method's.
POSE_DAG_OPS_PER_TEST = 497.0 / 16.0
# The same count for the 5-DoF predicate (32 children: the 4-DoF ones for
# each half of the cell's f interval): z bits 21; per f bit the slopes
# |eta| f_lo, |eta| f_hi and their squares (4, x2 = 8); kappa: padded ends
# (2) and per (kappa bit, f bit) the tangents' ends (1 product, 1 select of
# two shared per f bit) and edges (6): 34; (x, y) parts (4), 183 each: 39 as
# above plus 9 per (z bit, f bit) and 27 per (kappa bit, f bit); child
# masks 32.  827 operations for 32 tests.
POSE5_DAG_OPS_PER_TEST = 827.0 / 32.0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(g, budget_tests, threads):
    """The oracle as it stands, stopped after a fixed number of incidence
    tests of the same solve: on one host thread, and on `threads` threads
    (its thread pool over disjoint subtrees, same result)."""
    import oracle
    out = {}
    for nt in (threads, 1):
        pr = oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], test_budget=int(budget_tests * nt),
                            threads=nt)
        r = oracle.solve(pr)
        out[nt] = (r["tests"] / r["seconds"], r["tests"], r["seconds"])
    v, n, sec = out[threads]
    v1, n1, sec1 = out[1]
    return {"value": v, "unit": "tests/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n:.3g} incidence tests of the same solve (greedy dive then depth-first search over "
                      f"disjoint subtrees), {threads} host threads, {sec:.1f} s",
            "single_thread": {"value": v1, "cores": 1,
                              "sample": f"first {n1:.3g} incidence tests, one host thread, {sec1:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def single_leg(name, args, ctx, warmup, steps):
    """Timed solves of one workload with inputs resident in HBM: throughput,
    the roofline of the dominant kernel, and the comparison with the
    oracle's golden result."""
    from paper_2107_11810_amd import gvote, synth
    W = WORKLOADS[name]
    g = synth.config(name)
    cols = gvote.to_device(g["cols"])  # inputs resident in HBM
    hip = gvote.hip()

    def solve():
        return ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], precision=args.precision)

    for i in range(warmup):
        r = solve()
        print(f"{name} warmup {i}: count={r['count']} tests={r['stats']['tests']:.3g} "
              f"{r['stats']['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    hip.hipDeviceSynchronize()
    results = []
    t0 = time.perf_counter()
    for i in range(steps):
        results.append(solve())
    hip.hipDeviceSynchronize()
    sec = time.perf_counter() - t0
    for i, r in enumerate(results):
        print(f"{name} step {i}: count={r['count']} inliers={r['n_inliers']} tests={r['stats']['tests']:.3g} "
              f"{r['stats']['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    tests = sum(r["stats"]["tests"] for r in results)
    st = [r["stats"] for r in results]
    t_ms = sum(s["test_ms"] for s in st)
    c_ms = sum(s["compact_ms"] for s in st)
    t_b = sum(s["test_bytes"] for s in st)
    c_b = sum(s["compact_bytes"] for s in st)
    t_n = sum(s["test_launches"] for s in st)
    c_n = sum(s["compact_launches"] for s in st)
    c_wb = sum(s.get("compact_write_bytes", 0) for s in st)
    if t_ms >= c_ms:
        kname, kms, kb, kn = W["kernel"], t_ms, t_b, t_n
    else:
        kname, kms, kb, kn = W["compact"], c_ms, c_b, c_n
    achieved = (kb / kn) / (kms / kn * 1e-3) / 1e9 if kn and kms > 0 else 0.0
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, kname),
            "launches": kn, "avg_launch_us": round(kms / kn * 1e3, 2) if kn else None,
            "bytes_per_launch": int(kb / kn) if kn else None,
            "kernel_ms_per_step": round(kms / len(results), 2),
            "other_kernel_ms_per_step": round((c_ms if kname == W["kernel"] else t_ms) / len(results), 2),
            # both big kernels: the incidence test (count pass) and compaction
            "kernels": [per_kernel(W["kernel"], t_ms, t_b, t_n, len(results)),
                        per_kernel(W["compact"], c_ms, c_b, c_n, len(results))]}
    if c_ms > 0 and c_wb:
        # the same two kernels counted with each entry read once per expansion
        # (by the count pass) and written once (by the compaction): the
        # compaction's re-read of its parents is left out of its work
        roof["kernels"][1]["write_achieved"] = round(c_wb / (c_ms * 1e-3) / 1e9, 1)
        roof["kernels"][1]["write_frac"] = round(c_wb / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        pb = (t_b + c_wb) / (t_ms + c_ms) / 1e6 if t_ms + c_ms > 0 else 0.0
        roof["path"] = {"basis": "count-pass reads plus compaction child writes, over both kernels' time",
                        "bytes_per_step": int((t_b + c_wb) / len(results)),
                        "ms_per_step": round((t_ms + c_ms) / len(results), 2),
                        "achieved": round(pb, 1), "unit": "GB/s", "frac": round(pb / HBM_PEAK_GBS, 4)}
    for k, ms in zip(roof["kernels"], (t_ms, c_ms)):
        opt_k = measured_valu(name, k["kernel"])
        if opt_k is not None:
            k["valu_frac"] = valu_frac(opt_k, tests, ms)
    if W["bound"] == "alu" and kname == W["kernel"] and kms > 0:
        # the incidence kernel of this family is bound by vector ALU work:
        # operations per test of the predicate's definition, times the tests,
        # over its event time; beside it the measured issue rate (VALU
        # instructions x 64 lanes per test, from the counter record)
        opt = POSE5_DAG_OPS_PER_TEST if g["family"] == "pose5dof" else POSE_DAG_OPS_PER_TEST
        ach = opt * tests / (kms * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": round(ach, 2), "peak": VALU_LANE_OPS / 1e12,
                     "unit": "T ops/s", "frac": round(ach / (VALU_LANE_OPS / 1e12), 4),
                     "ops_per_test": round(opt, 2), "traffic": None})
        issued = measured_valu(name, kname)
        if issued is not None:
            roof["issued_lane_ops_per_test"] = round(issued, 2)
            roof["issue_frac"] = valu_frac(issued, tests, kms)
    gold = load_golden(name)
    golden = None
    if gold is not None:
        gg = gold["problems"][0]
        golden = {"matches": all(golden_match(r, gg) for r in results), "oracle_tests_per_solve": gg["oracle_tests"],
                  "oracle_wall_s": round(gg["oracle_wall_s"], 1), "oracle_threads": gold.get("threads"),
                  "oracle_solves_per_s": round(1.0 / gg["oracle_wall_s"], 6)}
    refine = None
    if g["family"] in ("pose4dof", "pose5dof"):
        refine = refine_leg(ctx, g, cols, results[0])
    for c in cols:
        c.free()
    return {
        "refine": refine,
        "g": g, "sec": sec, "steps": steps, "tests": tests, "results": results, "roofline": roof,
        "tests_per_s": tests / sec, "solves_per_s": steps / sec, "ms_per_solve": 1e3 * sec / steps,
        "tests_per_solve": tests / steps, "count": results[0]["count"],
        # each solve's own wall time, measured by the library (device-resident inputs to the result
        # in host memory): the median of the timed solves
        "ms_per_solve_median": median([r["stats"]["ms_total"] for r in results]),
        "deterministic": len({(r["count"], r["leaf_index"]) for r in results}) == 1, "golden": golden,
        "rechecks_per_solve": sum(r["stats"]["fp64_rechecks"] for r in results) / steps,
    }


def refine_leg(ctx, g, cols, vote, reps=5):
    """Verification and refinement after the vote (gv_refine) of a pose
    workload: time per call, matches kept, pose error before and after."""
    tau0, tau = math.radians(1.5), math.radians(0.75)
    args = (g["family"], cols, g["lo"], g["hi"], g["eps"], vote["leaf_index"], vote["inliers"], tau0, tau)
    r = ctx.refine(*args, rounds=3, iters=10)
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.refine(*args, rounds=3, iters=10)
    ms = 1e3 * (time.perf_counter() - t0) / reps
    tr = list(map(float, g["truth"]))

    def err(q):
        dyaw = abs(q[3] - tr[3])
        e = {"position_m": math.dist(q[:3], tr[:3]), "yaw_deg": math.degrees(min(dyaw, 2 * math.pi - dyaw))}
        if g["family"] == "pose5dof":
            e["f_rel"] = abs(q[4] - tr[4]) / tr[4]
        return {k: round(v, 6) for k, v in e.items()}

    return {"ms_per_refine": round(ms, 3), "rounds": 3, "iters": 10, "tau0_deg": 1.5, "tau_deg": 0.75,
            "vote_inliers": int(vote["n_inliers"]), "kept": int(len(r["verified"])), "rms0": r["rms0"],
            "rms": r["rms"], "error_leaf_centre": err(vote["point"]), "error_refined": err(r["pose"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=3, help="untimed solves first (they include the autotuning)")
    ap.add_argument("--workload", default="plane3d_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-tests", type=float, default=2.5e8, help="oracle sample size per thread (incidence tests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
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
    from paper_2107_11810_amd import gvote
    ok = True
    if args.workload == "pose4dof_serve256":
        sv = serve_bench(args)
        ok = sv["identical_to_plain"] and (sv["golden"] is None or sv["golden"]["matches"])
        out = {
            "metric": "solves/s", "value": sv["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": sv["n_problems"], "warmup": 1, "ms_per_step": sv["ms_batched"] / sv["n_problems"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": "pose4dof_serve256", "description": WORKLOADS["pose4dof_serve256"]["desc"],
                       "n_problems": sv["n_problems"], "total_matches": sv["total_matches"]},
        }
        out.update({k: v for k, v in sv.items() if k not in ("solves_per_s", "n_problems", "total_matches")})
        print(json.dumps(out), flush=True)
        sys.exit(0 if ok else 1)

    W = WORKLOADS[args.workload]
    ctx = gvote.Context(0, kernel_timing=True)
    head = single_leg(args.workload, args, ctx, args.warmup, args.steps)
    g = head["g"]
    n = len(g["cols"][0])
    out = {
        "metric": "incidence tests/s",
        "value": head["tests_per_s"],
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("int32" if g["family"] not in ("pose4dof", "pose5dof")
                  else ("f32+f64" if args.precision else "f64")),
        "data": "synthetic",
        "config": {"workload": args.workload, "description": W["desc"], "n": n, "eps": g["eps"],
                   "canon_c": 1.0,
                   # the linear families decide every test exactly on an integer lattice, so the
                   # precision setting (binary32 filter or binary64) applies to the pose families only
                   "precision": ("int32_lattice" if g["family"] not in ("pose4dof", "pose5dof")
                                 else ("fp32_filter" if args.precision else "fp64_plain"))},
        "solves_per_s": head["solves_per_s"],
        "ms_per_solve_median": round(head["ms_per_solve_median"], 3),
        "tests_per_solve": head["tests_per_solve"],
        "count": head["count"],
        "deterministic": head["deterministic"],
        "roofline": head["roofline"],
        "golden": head["golden"],
    }
    if head["golden"] is not None:
        ok = ok and head["golden"]["matches"]
    if args.workload == "plane3d_1m" and not args.no_extras:
        # the 4-DoF pose workload, timed the same way
        pl = single_leg("pose4dof_1m", args, ctx, 3, 10)
        out["pose4dof_1m"] = {
            "description": WORKLOADS["pose4dof_1m"]["desc"], "tests_per_s": pl["tests_per_s"],
            "ms_per_solve": pl["ms_per_solve"], "ms_per_solve_median": round(pl["ms_per_solve_median"], 3),
            "solves_per_s": pl["solves_per_s"],
            "tests_per_solve": pl["tests_per_solve"], "count": pl["count"], "roofline": pl["roofline"],
            "rechecks_per_solve": pl["rechecks_per_solve"], "golden": pl["golden"]}
        out["pose4dof_1m"]["refine"] = pl["refine"]
        if pl["golden"] is not None:
            ok = ok and pl["golden"]["matches"]
        # the 5-DoF pose workload (unknown focal length)
        p5 = single_leg("pose5dof_20k", args, ctx, 3, 10)
        out["pose5dof_20k"] = {
            "description": WORKLOADS["pose5dof_20k"]["desc"], "tests_per_s": p5["tests_per_s"],
            "ms_per_solve": p5["ms_per_solve"], "ms_per_solve_median": round(p5["ms_per_solve_median"], 3),
            "solves_per_s": p5["solves_per_s"],
            "tests_per_solve": p5["tests_per_solve"], "count": p5["count"], "roofline": p5["roofline"],
            "rechecks_per_solve": p5["rechecks_per_solve"], "golden": p5["golden"], "refine": p5["refine"]}
        if p5["golden"] is not None:
            ok = ok and p5["golden"]["matches"]
    # (the serving leg gets a context of its own, after this one has released
    # the device memory its caching allocator holds: a budget taken from the
    # free memory left beside the 1e6-point solves' cache made it 15% slower)
    ctx.close()
    if args.workload == "plane3d_1m" and not args.no_extras:
        # the serving workload: batched binary32 filter against plain binary64
        sv = serve_bench(args)
        out["pose4dof_serve256"] = dict({"description": WORKLOADS["pose4dof_serve256"]["desc"]}, **sv)
        ok = ok and sv["identical_to_plain"] and (sv["golden"] is None or sv["golden"]["matches"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_tests, max(1, min(os.cpu_count() or 1, 16)))
    out["matches_oracle"] = ok
    print(json.dumps(out), flush=True)
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
