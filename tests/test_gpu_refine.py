"""Device parity of the verification and refinement after the vote
(gv_refine; pose families) with the oracle, through the C ABI.

Bar:
  * the first verification (at the vote's leaf centre) involves no sum: the
    kept set is bit-equal and, with zero rounds, the pose is the leaf centre
    exactly;
  * after Gauss-Newton rounds the device sums the normal equations in a
    different order than the oracle, so poses agree to rounding: |dx|, |dy|,
    |dz| <= 1e-8 m, |d yaw| <= 1e-10 rad, |df| <= 1e-10 (5-DoF) and the rms
    to 1e-8 relative (binary64 sums of at most ~1e4 terms of size ~1, damped
    5x5 systems with condition numbers below 1e4 here: differences of order
    1e-12).  The kept sets at the final pose are equal wherever a match's
    angle test is not within 1e-9 (relative) of its threshold, which the
    test checks holds for all but at most one match.
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


def margins(g, pose, sector, idx, tau):
    """Relative margin of the angle test |o x d|^2 <= tan^2(tau) (o.d)^2 at a
    pose given in the sector's frame (x, y, z, kappa[, f])."""
    x, y, z, k = pose[:4]
    f = pose[4] if g["family"] == "pose5dof" else 1.0
    w1, w2, w3, xi, eta = (np.asarray(c)[idx] for c in g["cols"])
    a, b = xi * f, eta * f
    o = np.stack([np.ones_like(a), a, b * np.sqrt(1 + a * a)], axis=1)
    A, B = w1 - x, w2 - y
    u1, u2 = [(A, B), (B, -A), (-A, -B), (-B, A)][sector]
    n = math.sqrt(1 + k * k)
    d = np.stack([(u1 + k * u2) / n, (u2 - k * u1) / n, w3 - z], axis=1)
    dot = np.sum(o * d, axis=1)
    cr = np.sum(np.cross(o, d) ** 2, axis=1)
    T2 = math.tan(tau) ** 2
    return np.abs(cr - T2 * dot * dot) / np.maximum(cr + T2 * dot * dot, 1e-300)


def sector_frame(pose, sector):
    q = list(pose)
    q[3] = math.tan(q[3] - sector * math.pi / 2)
    return q


def check_close(g, rg, ro, r_vote, tau):
    d = 5 if g["family"] == "pose5dof" else 4
    for j in range(3):
        assert abs(rg["pose"][j] - ro["pose"][j]) <= 1e-8, (j, rg["pose"][j], ro["pose"][j])
    dy = abs(rg["pose"][3] - ro["pose"][3])
    assert min(dy, 2 * math.pi - dy) <= 1e-10
    if d == 5:
        assert abs(rg["pose"][4] - ro["pose"][4]) <= 1e-10
    assert abs(rg["rms"] - ro["rms"]) <= 1e-8 * max(ro["rms"], 1e-12)
    assert abs(rg["rms0"] - ro["rms0"]) <= 1e-12 * max(ro["rms0"], 1e-12)
    m = margins(g, sector_frame(ro["pose"], r_vote["sector"]), r_vote["sector"], r_vote["inliers"], tau)
    clear = m > 1e-9
    assert np.sum(~clear) <= 1
    kg = np.isin(r_vote["inliers"], rg["verified"])
    ko = np.isin(r_vote["inliers"], ro["verified"])
    assert np.array_equal(kg[clear], ko[clear])


CASES = [("pose4dof_small", 14), ("pose4dof_small", 16), ("pose4dof_small_flat", 18), ("pose5dof_small", 17),
         ("pose5dof_small", 23), ("pose5dof_tiny", 7), ("pose5dof_20k", None), ("pose4dof_tiny", 2)]


@pytest.mark.parametrize("name,seed", CASES)
def test_refine_equals_oracle(ctx, name, seed):
    g = synth.config(name) if seed is None else synth.config(name, seed=seed)
    pr = OP(g)
    rv = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    tau0, tau = math.radians(4.0), math.radians(1.5)
    if name == "pose5dof_20k":
        tau0, tau = math.radians(1.5), math.radians(0.75)
    _say("refine", name, seed, "vote inliers", rv["n_inliers"])
    # zero rounds: the verification at the leaf centre alone, bit-exact
    r0 = ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"], rv["inliers"], tau0, tau,
                    rounds=0)
    o0 = oracle.refine(pr, rv["leaf_index"], rv["inliers"], tau0, tau, rounds=0)
    assert np.array_equal(r0["verified"], o0["verified"])
    assert r0["pose"] == o0["pose"]
    assert abs(r0["rms"] - o0["rms"]) <= 1e-12 * max(o0["rms"], 1e-12)  # (a sum: order differs)
    for rounds, iters in ((1, 6), (3, 10)):
        rg = ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"], rv["inliers"], tau0,
                        tau, rounds=rounds, iters=iters)
        ro = oracle.refine(pr, rv["leaf_index"], rv["inliers"], tau0, tau, rounds=rounds, iters=iters)
        _say("  rounds", rounds, "kept", len(rg["verified"]), "rms0 %.3g rms %.3g" % (rg["rms0"], rg["rms"]))
        check_close(g, rg, ro, rv, tau)


def test_refine_device_columns_and_edges(ctx):
    from paper_2107_11810_amd import gvote
    g = synth.config("pose5dof_small")
    rv = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    dcols = gvote.to_device(g["cols"])
    a = ctx.refine(g["family"], dcols, g["lo"], g["hi"], g["eps"], rv["leaf_index"], rv["inliers"], 0.07, 0.03)
    b = ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"], rv["inliers"], 0.07, 0.03)
    assert a["pose"] == b["pose"] and np.array_equal(a["verified"], b["verified"])  # deterministic
    # no matches: the leaf centre, nothing kept
    e = ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"], np.zeros(0, np.int64),
                   0.07, 0.03)
    assert len(e["verified"]) == 0 and e["rms"] == 0.0
    assert e["pose"][:3] == rv["point"][:3] and e["pose"][4] == rv["point"][4]
    for bad in (dict(tau0=0.0), dict(tau=2.0)):
        kw = dict(tau0=0.07, tau=0.03)
        kw.update(bad)
        with pytest.raises(gvote.GvError):
            ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"], rv["inliers"], **kw)
    with pytest.raises(gvote.GvError):
        ctx.refine(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], rv["leaf_index"],
                   np.array([len(g["cols"][0])]), 0.07, 0.03)
    gl = synth.config("line2d_tiny")
    with pytest.raises(gvote.GvError):
        ctx.refine(gl["family"], gl["cols"], gl["lo"], gl["hi"], gl["eps"], 0, np.array([0]), 0.07, 0.03)
