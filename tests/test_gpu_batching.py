"""Batched solving and continuous batching through gv_submit / gv_poll.

Every result must be identical to the same problem solved alone (and to the
oracle), whatever mix of problems it shares the device with.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["solo_epochs", "shared_epochs"])
def ctx(request):
    """Default serving (one problem per epoch) and epochs shared by many
    problems (GV_BATCH_N read when the context is created)."""
    import os
    from paper_2107_11810_amd import gvote
    old = os.environ.get("GV_BATCH_N")
    if request.param == "shared_epochs":
        os.environ["GV_BATCH_N"] = "1000000"
    c = gvote.Context(0)
    if old is None:
        os.environ.pop("GV_BATCH_N", None)
    else:
        os.environ["GV_BATCH_N"] = old
    yield c
    c.close()


def same(a, b):
    return (a["count"] == b["count"] and a["leaf_index"] == b["leaf_index"] and a["sector"] == b["sector"]
            and np.array_equal(a["inliers"], b["inliers"]) and a["point"] == b["point"])


def pose_batch(k, seed0=500, nmin=300, nmax=6000):
    out = []
    for i in range(k):
        r = np.random.default_rng(seed0 + i)
        n = int(np.exp(r.uniform(np.log(nmin), np.log(nmax))))
        n_in = max(3, int(n * np.exp(r.uniform(np.log(0.02), np.log(0.2)))))
        out.append(synth.pose4dof(seed=seed0 + i, n=n, n_in=n_in, noise_deg=0.2, eps_m=4.0, eps_deg=2.0,
                                  rho_max=80.0))
    return out


def test_batch_equals_alone_and_oracle_pose(ctx):
    from paper_2107_11810_amd import gvote
    probs = pose_batch(12)
    _say("submit", len(probs))
    alone = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    tickets = [gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    for g, t, a in zip(probs, tickets, alone):
        st, r = gvote.poll(ctx, t, len(g["cols"][0]))
        assert st == 0
        assert same(r, a)
    for g, a in zip(probs[:4], alone[:4]):
        o = oracle.solve(oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]))
        assert (a["count"], a["leaf_index"]) == (o["count"], o["leaf_index"])
        assert np.array_equal(a["inliers"], o["inliers"])


@pytest.mark.parametrize("fam", ["line2d", "plane3d", "ray3d"])
def test_batch_linear_families(ctx, fam):
    from paper_2107_11810_amd import gvote
    probs = [synth.config(fam + "_small", seed=s) for s in (31, 32, 33, 34)]
    probs += [synth.config(fam + "_tiny", seed=s) for s in (1, 2)]
    _say("linear batch", fam)
    alone = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    tickets = [gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    for g, t, a in zip(probs, tickets, alone):
        st, r = gvote.poll(ctx, t, len(g["cols"][0]))
        assert st == 0
        assert same(r, a)


def test_mix_order_and_arrivals(ctx):
    """Results do not depend on which problems share an epoch or when they
    arrive: the same problems in three orders and with staggered arrivals."""
    from paper_2107_11810_amd import gvote
    probs = pose_batch(8, seed0=700)
    ref = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    rng = np.random.default_rng(3)
    for trial in range(3):
        order = rng.permutation(len(probs))
        tickets = {}
        for j, i in enumerate(order):
            g = probs[i]
            tickets[i] = gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
            if trial == 2 and j % 2 == 1:
                time.sleep(0.002)  # staggered arrivals join later epochs
        for i, t in tickets.items():
            st, r = gvote.poll(ctx, t, len(probs[i]["cols"][0]))
            assert st == 0 and same(r, ref[i])


def test_serving_error_paths(ctx):
    from paper_2107_11810_amd import gvote
    g = synth.config("line2d_small")
    # inlier buffer too small: the required size comes back, the ticket stays
    t = gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    st, r = gvote.poll(ctx, t, 2)
    assert st == -4 and r["n_inliers"] > 2
    st, r2 = gvote.poll(ctx, t, r["n_inliers"])
    assert st == 0 and r2["n_inliers"] == r["n_inliers"]
    # unknown ticket
    st, _ = gvote.poll(ctx, 999999, 10, timeout_ms=0)
    assert st == -1
    # invalid problem is rejected at submit
    bad = [np.array([0.3, np.inf]), np.array([0.2, 0.1])]
    t = gvote.submit(ctx, "line2d", bad, g["lo"], g["hi"], g["eps"])
    st, _ = gvote.poll(ctx, t, 10)
    assert st == -1
    # cancel: a cancelled ticket reports GV_ECANCELED (or finished first)
    big = synth.config("plane3d_small")
    ts = [gvote.submit(ctx, big["family"], big["cols"], big["lo"], big["hi"], big["eps"]) for _ in range(6)]
    assert gvote.cancel(ctx, ts[-1]) == 0
    for t in ts[:-1]:
        st, _ = gvote.poll(ctx, t, len(big["cols"][0]))
        assert st == 0
    st, _ = gvote.poll(ctx, ts[-1], len(big["cols"][0]))
    assert st in (0, -7)


def test_solve_while_serving(ctx):
    """gv_solve on the context's stream while the serving lanes run submitted
    problems: both give the results of solving each problem alone."""
    import threading
    from paper_2107_11810_amd import gvote
    probs = pose_batch(10, seed0=900)
    lin = [synth.config("plane3d_small", seed=s) for s in (51, 52, 53)]
    ref = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    ref_lin = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in lin]
    _say("serving while solving")
    tickets = [gvote.submit(ctx, g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in probs]
    out = {}

    def solver():
        out["lin"] = [ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]) for g in lin]
    th = threading.Thread(target=solver)
    th.start()
    for g, t, a in zip(probs, tickets, ref):
        st, r = gvote.poll(ctx, t, len(g["cols"][0]))
        assert st == 0 and same(r, a)
    th.join()
    for r, a in zip(out["lin"], ref_lin):
        assert same(r, a)
