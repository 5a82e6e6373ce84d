"""Write the oracle's results for the full-size workloads (golden files).

Calls only the CPU oracle (oracle/) and the seeded input generators; the
device path is never involved.  Each file holds, per problem: count, leaf
index, sector, leaf coordinates, number of inliers and the SHA-256 of the
sorted inlier indices (int64, little endian), the binary64 point, and the
oracle's own test count and time, plus the SHA-256 of the input columns so
that a change of the generator is detected.

    python tests/golden/make_golden.py plane3d_1m [--threads 8]
    python tests/golden/make_golden.py pose4dof_1m
    python tests/golden/make_golden.py pose4dof_serve256
    python tests/golden/make_golden.py pose5dof_20k
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2107_11810_amd import synth  # noqa: E402


def cols_sha(g):
    h = hashlib.sha256()
    for c in g["cols"]:
        h.update(np.ascontiguousarray(c, dtype="<f8").tobytes())
    return h.hexdigest()


def inliers_sha(inl):
    return hashlib.sha256(np.ascontiguousarray(np.sort(inl), dtype="<i8").tobytes()).hexdigest()


def truth_leaf(g):
    """Leaf holding the generator's planted truth (input metadata, not a
    result): its count by the oracle's replay is an achieved key, a valid
    starting bound that cannot change the result."""
    k = oracle.constants(oracle.Problem(g["family"], [np.zeros(0)] * len(g["cols"]), g["lo"], g["hi"], g["eps"]))
    tr = [float(x) for x in g["truth"]]
    if g["family"] in ("pose4dof", "pose5dof"):
        yaw = tr[3]
        s = int(math.floor((yaw + math.pi / 4) / (math.pi / 2))) % 4
        kap = math.tan(yaw - s * math.pi / 2)
        u = [(tr[j] - g["lo"][j]) / (g["hi"][j] - g["lo"][j]) for j in range(3)] + [(kap + 1) / 2]
        if g["family"] == "pose5dof":
            u.append((tr[4] - g["lo"][4]) / (g["hi"][4] - g["lo"][4]))
        d = len(u)
    else:
        s = None
        d = len(g["lo"])
        u = [(tr[j] - g["lo"][j]) / (g["hi"][j] - g["lo"][j]) for j in range(d)]
    L = k["L"][:d]
    coords = [min(2 ** L[j] - 1, max(0, int(math.floor(u[j] * 2 ** L[j])))) for j in range(d)]
    return oracle.leaf_index_of(L, coords, s)


def solve_one(g, threads):
    pr = oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], threads=threads, seed_leaf=truth_leaf(g))
    t0 = time.perf_counter()
    r = oracle.solve(pr)
    wall = time.perf_counter() - t0
    return {
        "n": int(len(g["cols"][0])), "cols_sha256": cols_sha(g),
        "count": int(r["count"]), "leaf_index": int(r["leaf_index"]), "sector": int(r["sector"]),
        "leaf_coords": [int(x) for x in r["leaf_coords"]], "n_inliers": int(r["n_inliers"]),
        "inliers_sha256": inliers_sha(r["inliers"]), "point": [float(x) for x in r["point"]],
        "oracle_tests": int(r["tests"]), "oracle_search_s": float(r["seconds"]), "oracle_wall_s": wall,
        "seed_leaf": int(pr.seed_leaf),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["line2d_10k", "ray3d_100k", "plane3d_1m", "pose4dof_1m",
                                         "pose4dof_serve256", "pose5dof_20k"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    out = {"workload": args.workload, "threads": args.threads, "host_cpus": os.cpu_count(),
           "cpu_model": platform.processor() or "", "problems": []}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                out["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    probs = synth.batch_pose4dof(n_problems=256) if args.workload == "pose4dof_serve256" \
        else [synth.config(args.workload)]
    t0 = time.perf_counter()
    for i, g in enumerate(probs):
        rec = solve_one(g, args.threads)
        out["problems"].append(rec)
        print(f"{args.workload} #{i}: n={rec['n']} count={rec['count']} leaf={rec['leaf_index']} "
              f"tests={rec['oracle_tests']:.3g} {rec['oracle_wall_s']:.1f} s", flush=True)
    out["total_wall_s"] = time.perf_counter() - t0
    path = os.path.join(HERE, f"{args.workload}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print(path)


if __name__ == "__main__":
    main()
