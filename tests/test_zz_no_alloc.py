"""gv_solve_noalloc (the entry point for callers that cannot allocate)
against gv_solve: identical results on consecutive calls, the second with a
smaller input; host and device columns; the size limit; and no device
memory taken by the calls themselves."""
import ctypes
import math
import sys

import numpy as np
import pytest

from paper_2107_11810_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    return (a["count"] == b["count"] and a["leaf_index"] == b["leaf_index"] and a["sector"] == b["sector"]
            and np.array_equal(a["inliers"], b["inliers"]) and a["point"] == b["point"]
            and a["bound"] == b["bound"])


@pytest.fixture(scope="module")
def ctx():
    from paper_2107_11810_amd import gvote
    c = gvote.Context(0)
    yield c
    c.close()


def _free_bytes():
    from paper_2107_11810_amd import gvote
    H = gvote.hip()
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    H.hipMemGetInfo.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    H.hipMemGetInfo.restype = ctypes.c_int
    assert H.hipMemGetInfo(ctypes.byref(f), ctypes.byref(t)) == 0
    return f.value


SEQ = [
    ("pose4dof", lambda: synth.pose4dof(seed=10032, n=175_000, n_in=1200)),
    ("pose4dof", lambda: synth.config("pose4dof_small")),
    ("plane3d", lambda: synth.plane3d(seed=7, n=120_000, n_in=3000, eps=(0.01, 0.01, 0.01))),
    ("plane3d", lambda: synth.config("plane3d_small")),
    ("line2d", lambda: synth.config("line2d_10k")),
    ("line2d", lambda: synth.config("line2d_tiny")),
    ("ray3d", lambda: synth.config("ray3d_small")),
    ("ray3d", lambda: synth.config("ray3d_tiny")),
]


@pytest.mark.parametrize("k", range(0, len(SEQ), 2))
def test_noalloc_equals_solve_twice_in_a_row(ctx, k):
    """Two allocation-free solves in a row, the second smaller: each equals
    gv_solve on the same input (bit for bit)."""
    for j in (k, k + 1):
        fam, make = SEQ[j]
        g = make()
        _say("noalloc", fam, len(g["cols"][0]))
        ref = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
        got = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], noalloc=True)
        assert same(got, ref)


def test_noalloc_device_columns_exact_mode_and_limits(ctx):
    from paper_2107_11810_amd import gvote
    g = synth.config("ray3d_100k")
    cols = gvote.to_device(g["cols"])
    ref = ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"])
    for _ in range(2):
        assert same(ctx.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], noalloc=True), ref)
    g = synth.config("plane3d_tiny", seed=2)
    ref = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf)
    assert same(ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf, noalloc=True), ref)
    # beyond the size limit: refused before any work
    n = (1 << 19) + 1
    big = [np.random.default_rng(1).uniform(0, 1, n) for _ in range(2)]
    with pytest.raises(gvote.GvError) as e:
        ctx.solve("line2d", big, [-1, -1], [1, 2], [0.005, 0.005], noalloc=True)
    assert e.value.status == -3
    # and the context still works
    g = synth.config("line2d_small")
    ref = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    assert same(ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], noalloc=True), ref)


def test_noalloc_takes_no_device_memory():
    """In a fresh context, allocation-free solves leave the free device
    memory unchanged (inputs already resident)."""
    from paper_2107_11810_amd import gvote
    c = gvote.Context(0)
    try:
        g = synth.pose4dof(seed=10077, n=60_000, n_in=900)
        cols = gvote.to_device(g["cols"])
        first = c.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], noalloc=True)
        gvote.hip().hipDeviceSynchronize()
        f0 = _free_bytes()
        for _ in range(3):
            r = c.solve(g["family"], cols, g["lo"], g["hi"], g["eps"], noalloc=True)
            assert same(r, first)
        gvote.hip().hipDeviceSynchronize()
        f1 = _free_bytes()
        _say("free bytes before/after", f0, f1)
        assert f1 == f0
    finally:
        c.close()
