"""Device results at the full benchmark sizes, in the configuration bench.py
times (default context, binary32 filter, inputs resident in device memory).

ray3d_100k and line2d_10k: the oracle's full search finishes in seconds, so
the comparison is run here.  plane3d_1m, pose4dof_1m and the 256 problems
of pose4dof_serve256: complete comparison with golden files that a
committed script wrote from the oracle alone (tests/golden/make_golden.py):
count, leaf, sector, leaf coordinates, point and the SHA-256 of the sorted
inlier set, per problem; the served problems go through gv_submit/gv_poll.
Also, for the two large single problems, the oracle's replay of the chosen
leaf and the planted-inlier lower bound.
"""
import hashlib
import json
import os
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2107_11810_amd import gvote
    c = gvote.Context(0)
    yield c
    c.close()


def OP(g, **kw):
    return oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], **kw)


def solve_dev(ctx, g):
    from paper_2107_11810_amd import gvote
    cols = gvote.to_device(g["cols"])
    r = ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], precision=gvote.FP32_FILTER)
    for c in cols:
        c.free()
    return r


def key(count, idx, B):
    return (count << B) | ((1 << B) - 1 - idx)


def truth_coords(g, k):
    fam = g["family"]
    tr = list(map(float, g["truth"]))
    if fam == "pose4dof":
        s = int(math.floor((tr[3] + math.pi / 4) / (math.pi / 2))) % 4
        kap = math.tan(tr[3] - s * math.pi / 2)
        u = [(tr[j] - g["lo"][j]) / (g["hi"][j] - g["lo"][j]) for j in range(3)] + [(kap + 1) / 2]
        d = 4
    else:
        s = None
        d = len(g["lo"])
        u = [(tr[j] - g["lo"][j]) / (g["hi"][j] - g["lo"][j]) for j in range(d)]
    L = k["L"][:d]
    return [min(2 ** L[j] - 1, max(0, int(math.floor(u[j] * 2 ** L[j])))) for j in range(d)], s


def leaf_idx(k, coords, sector):
    d = len(coords)
    return oracle.leaf_index_of(k["L"][:d], coords, sector)


@pytest.mark.parametrize("name", ["line2d_10k", "ray3d_100k"])
def test_fullsize_complete_parity(ctx, name):
    g = synth.config(name)
    _say("full", name)
    r = solve_dev(ctx, g)
    o = oracle.solve(OP(g))
    assert (r["count"], r["leaf_index"], r["sector"]) == (o["count"], o["leaf_index"], o["sector"])
    assert np.array_equal(r["inliers"], o["inliers"])
    assert r["point"][:3] == o["point"][:3]


@pytest.mark.parametrize("name", ["plane3d_1m", "pose4dof_1m"])
def test_fullsize_sampled_parity(ctx, name):
    g = synth.config(name)
    pr = OP(g)
    k = oracle.constants(pr)
    B = k["B"]
    _say("full-size", name)
    r = solve_dev(ctx, g)
    best = key(r["count"], r["leaf_index"], B)
    # 1. the chosen leaf: same count and the same sorted inlier set by replay
    c, inl = oracle.leaf_count(pr, r["leaf_index"], with_inliers=True)
    assert c == r["count"]
    assert np.array_equal(inl, r["inliers"])
    # 2. no sampled leaf beats it: the truth's leaf, its neighbours, random leaves
    tc, s = truth_coords(g, k)
    d = len(tc)
    L = k["L"][:d]
    rng = np.random.default_rng(5)
    cand = [tc]
    for j in range(d):
        for dd in (-1, 1):
            cc = list(tc)
            cc[j] = min(2 ** L[j] - 1, max(0, cc[j] + dd))
            cand.append(cc)
    wc = r["leaf_coords"][:d]
    for j in range(d):
        for dd in (-1, 1):
            cc = list(wc)
            cc[j] = min(2 ** L[j] - 1, max(0, cc[j] + dd))
            cand.append(cc)
    for _ in range(6):
        cand.append([int(rng.integers(0, 2 ** L[j])) for j in range(d)])
    sectors = [s] if s is not None else [None]
    if s is not None:
        sectors.append(r["sector"])
    for cc in cand:
        for sec in sectors:
            idx = leaf_idx(k, cc, sec)
            cnt = oracle.leaf_count(pr, idx)
            assert key(cnt, idx, B) <= best, (cc, sec, cnt)
    # 3. planted lower bound: every observation within eps of the truth counts
    # at the truth's leaf, and the maximum is at least that
    idx_t = leaf_idx(k, tc, s)
    ct = oracle.leaf_count(pr, idx_t)
    planted_in = len(set(r["inliers"].tolist()) & set(g["planted"].tolist()))
    _say(f"  count {r['count']} truth-leaf {ct} planted found {planted_in}/{len(g['planted'])}")
    assert r["count"] >= ct
    assert planted_in >= 0.8 * len(g["planted"])


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"no golden file for {name}")
    return json.load(open(path))


def _cols_sha(g):
    h = hashlib.sha256()
    for c in g["cols"]:
        h.update(np.ascontiguousarray(c, dtype="<f8").tobytes())
    return h.hexdigest()


def _inl_sha(inl):
    return hashlib.sha256(np.ascontiguousarray(np.sort(inl), dtype="<i8").tobytes()).hexdigest()


def _axes(v, n):
    """The first n per-axis values; the rest (axes the family lacks) are 0."""
    v = list(v)
    assert all(x == 0 for x in v[n:])
    return v[:n]


def check_golden(r, gold):
    assert r["count"] == gold["count"], (r["count"], gold["count"])
    assert r["leaf_index"] == gold["leaf_index"]
    assert r["sector"] == gold["sector"]
    assert _axes(r["leaf_coords"], len(gold["leaf_coords"])) == gold["leaf_coords"]
    assert r["n_inliers"] == gold["n_inliers"]
    assert _inl_sha(r["inliers"]) == gold["inliers_sha256"]
    assert [float(x) for x in _axes(r["point"], len(gold["point"]))] == gold["point"]


@pytest.mark.parametrize("name", ["plane3d_1m", "pose4dof_1m", "pose5dof_20k"])
def test_fullsize_golden_parity(ctx, name):
    gold = _golden(name)["problems"][0]
    g = synth.config(name)
    assert _cols_sha(g) == gold["cols_sha256"]  # the generator has not changed
    _say("golden", name)
    for prec in (1, 0):
        from paper_2107_11810_amd import gvote
        cols = gvote.to_device(g["cols"])
        r = ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], precision=prec)
        _say(f"  precision {prec}: count {r['count']} tests {r['stats']['tests']:.3g} "
             f"(oracle {gold['oracle_tests']:.3g})")
        check_golden(r, gold)


def test_serve256_golden_parity(ctx):
    """All 256 problems of the serving workload through continuous batching
    (and the binary64 plain form for every eighth) against their goldens."""
    from paper_2107_11810_amd import gvote
    gold = _golden("pose4dof_serve256")["problems"]
    probs = synth.batch_pose4dof(n_problems=256)
    assert len(gold) == len(probs)
    _say("serve256 golden")
    cols = [gvote.to_device(g["cols"]) for g in probs]
    tickets = [gvote.submit(ctx, g["family"], c, g["lo"], g["hi"], g["eps"]) for g, c in zip(probs, cols)]
    for i, (g, t) in enumerate(zip(probs, tickets)):
        st, r = gvote.poll(ctx, t, len(g["cols"][0]))
        assert st == 0, (i, st)
        assert _cols_sha(g) == gold[i]["cols_sha256"], i
        check_golden(r, gold[i])
    for i in range(0, len(probs), 8):
        g = probs[i]
        r = ctx.solve(g["family"], cols[i], g["lo"], g["hi"], g["eps"], precision=gvote.FP64_PLAIN)
        check_golden(r, gold[i])
