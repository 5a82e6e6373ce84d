"""Device parity of the 5-DoF camera-posing family (Sec. 4.2.1: known
gravity, unknown focal length; axes x, y, z, yaw, f) with the oracle,
through the C ABI.

Bar: bit-exact front-end parameters; bit-exact count, leaf index, sector,
leaf coordinates, sorted inliers and binary64 point; pass masks of single
cells bit-equal; threshold reports equal; results the same alone, batched
and through the allocation-free entry point.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2107_11810_amd import gvote
    c = gvote.Context(0)
    yield c
    c.close()


def OP(g, **kw):
    return oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], **kw)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_same(r_gpu, r_or):
    assert r_gpu["count"] == r_or["count"], (r_gpu["count"], r_or["count"])
    assert r_gpu["leaf_index"] == r_or["leaf_index"]
    assert r_gpu["sector"] == r_or["sector"]
    assert r_gpu["n_inliers"] == r_or["n_inliers"]
    assert np.array_equal(r_gpu["inliers"], r_or["inliers"])
    assert list(r_gpu["leaf_coords"]) == list(r_or["leaf_coords"])
    for j in range(5):
        assert r_gpu["point"][j] == r_or["point"][j]  # bit-equal binary64


def solve(ctx, g, **kw):
    return ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], **kw)


@pytest.mark.parametrize("name", ["pose5dof_small", "pose5dof_tiny", "pose5dof_20k"])
def test_front_end_bit_exact(ctx, name):
    g = synth.config(name)
    _say("front", name)
    t, f, tag = ctx.parametrize(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    to, fo, tago = oracle.parametrize(OP(g))
    assert np.array_equal(t.view(np.uint64), to.view(np.uint64))
    assert np.array_equal(f.view(np.uint64), fo.view(np.uint64))


@pytest.mark.parametrize("seed", [7, 8, 9, 10, 11])
def test_tiny_parity(ctx, seed):
    g = synth.config("pose5dof_tiny", seed=seed)
    _say("tiny", seed)
    ro = oracle.solve(OP(g))
    for prec in (0, 1):
        check_same(solve(ctx, g, precision=prec), ro)


@pytest.mark.parametrize("seed", [17, 19, 21])
def test_small_parity(ctx, seed):
    g = synth.config("pose5dof_small", seed=seed)
    _say("small", seed)
    ro = oracle.solve(OP(g, threads=4))
    for prec in (0, 1):
        check_same(solve(ctx, g, precision=prec), ro)


def test_incidence_masks_equal_the_oracle(ctx):
    """gv_incidence against the oracle's cell masks at random cells of every
    level (up to 32 children), in both modes and in exact mode."""
    rng = np.random.default_rng(43)
    for name in ("pose5dof_small", "pose5dof_tiny"):
        g = synth.config(name)
        for c in (0.0, math.inf):
            pr = OP(g, canon_c=c)
            k = oracle.constants(pr)
            L, Ls = k["L"], k["Lstar"]
            for _ in range(6):
                m = int(rng.integers(0, Ls))
                cc = [int(rng.integers(0, 2 ** min(m, L[j]))) for j in range(5)]
                sec = int(rng.integers(0, 4))
                _say("incidence", name, c, m, sec, cc)
                mo = oracle.cell_masks(pr, m, sec, cc)
                for prec in (0, 1):
                    mg, tests, _ = ctx.incidence(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], m, sec, cc,
                                                 canon_c=c, precision=prec)
                    assert np.array_equal(mg, mo), (m, sec, cc, prec, int(np.sum(mg != mo)))
                    assert tests == g["cols"][0].size << sum(1 for j in range(5) if m < L[j])


@pytest.mark.parametrize("seed", [7, 8])
def test_exact_mode_parity(ctx, seed):
    g = synth.config("pose5dof_tiny", seed=seed)
    _say("exact", seed)
    ro = oracle.solve(OP(g, canon_c=math.inf))
    check_same(solve(ctx, g, canon_c=math.inf), ro)


def test_report_equals_oracle(ctx):
    g = synth.config("pose5dof_small")
    pr = OP(g)
    best = oracle.solve(pr)["count"]
    tau = max(1, int(best * 0.6))
    li, lc = oracle.report(pr, tau)
    _say("report", tau, len(li))
    gi, gc, _ = ctx.report(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], tau)
    assert np.array_equal(gi, li) and np.array_equal(gc, lc)
    assert len(li) > 1


def test_batched_and_noalloc_equal_alone(ctx):
    from paper_2107_11810_amd import gvote
    probs = [synth.config("pose5dof_small", seed=s, n=n) for s, n in ((17, 3000), (23, 800), (29, 1500))] + \
        [synth.config("pose5dof_tiny", seed=s) for s in (7, 8)]
    alone = [solve(ctx, g) for g in probs]
    tickets = [gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    for g, t, a in zip(probs, tickets, alone):
        st, r = gvote.poll(ctx, t, len(g["cols"][0]), timeout_ms=60000)
        assert st == 0
        check_same(r, a)
    for g, a in zip(probs, alone):
        check_same(solve(ctx, g, noalloc=True), a)
    check_same(alone[1], oracle.solve(OP(probs[1])))


def test_every_inlier_within_the_reported_bound(ctx):
    """Each reported inlier's z range over the leaf's (x, y, f) box comes
    within bound[2] of the leaf's z interval (direct binary64 evaluation of
    its observation)."""
    g = synth.config("pose5dof_small")
    r = solve(ctx, g)
    lo, hi = g["lo"], g["hi"]
    E = [hi[j] - lo[j] for j in range(5)]
    k = oracle.constants(OP(g))
    L = k["L"]
    box = []
    for j in (0, 1, 2, 4):
        h = E[j] * 2.0 ** -L[j]
        box.append((lo[j] + r["leaf_coords"][j] * h, lo[j] + (r["leaf_coords"][j] + 1) * h))
    (x0, x1), (y0, y1), (z0, z1), (f0, f1) = box
    w1, w2, w3, xi, eta = (c[r["inliers"]] for c in g["cols"])
    dx = np.maximum(0.0, np.maximum(x0 - w1, w1 - x1))
    dy = np.maximum(0.0, np.maximum(y0 - w2, w2 - y1))
    rmin = np.hypot(dx, dy)
    rmax = np.hypot(np.maximum(np.abs(w1 - x0), np.abs(w1 - x1)), np.maximum(np.abs(w2 - y0), np.abs(w2 - y1)))
    prods = np.stack([eta * f0 * rmin, eta * f0 * rmax, eta * f1 * rmin, eta * f1 * rmax])
    zmin, zmax = w3 - prods.max(0), w3 - prods.min(0)
    zd = np.maximum(0.0, np.maximum(z0 - zmax, zmin - z1))
    assert r["n_inliers"] > 0 and np.all(zd <= r["bound"][2] * (1 + 1e-9))
    assert r["bound"][4] == 0.5 * E[4] * 2.0 ** -L[4]


def test_edge_cases(ctx):
    from paper_2107_11810_amd import gvote
    g = synth.config("pose5dof_small")
    empty = [c[:0] for c in g["cols"]]
    r = ctx.solve(g["family"], empty, g["lo"], g["hi"], g["eps"])
    assert r["count"] == 0 and r["n_inliers"] == 0
    one = [c[:1] for c in g["cols"]]
    check_same(ctx.solve(g["family"], one, g["lo"], g["hi"], g["eps"]),
               oracle.solve(oracle.Problem(g["family"], one, g["lo"], g["hi"], g["eps"])))
    # f must stay positive over the box
    bad_lo = list(g["lo"])
    bad_lo[4] = 0.0
    with pytest.raises(gvote.GvError):
        ctx.solve(g["family"], g["cols"], bad_lo, g["hi"], g["eps"])
    # image coordinates too wide for the f range: rejected like the oracle
    wide = [c.copy() for c in g["cols"]]
    wide[3][0] = 40.0
    with pytest.raises(gvote.GvError):
        ctx.solve(g["family"], wide, g["lo"], g["hi"], g["eps"])
    with pytest.raises(oracle.OracleError):
        oracle.solve(oracle.Problem(g["family"], wide, g["lo"], g["hi"], g["eps"]))
