"""Launch-shape autotuner: launch grids and surface tiles.

The count and compaction kernels loop over list items, so their grid and the
number of entries per item (the count pass's surface tile) change nothing but
speed: results with the autotuner trying its candidates, with every fixed
grid and tile, and with choices read back from the cache file are all
identical, and equal to the oracle's.  The cache file holds one valid line
per tuned (family, choice): 0 count grid, 1 compaction grid, 2 count tile.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth

pytestmark = pytest.mark.gpu

CANDIDATES = {2, 4, 8, 16, 32}
TILE_LOGS = {8, 9, 10}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Env:
    """Environment knobs set for the block (read when a context is created
    and when an epoch starts, so they stay set while the context solves)."""
    def __init__(self, **kv):
        self.kv = kv
        self.old = {}

    def __enter__(self):
        for k, v in self.kv.items():
            self.old[k] = os.environ.get(k)
            os.environ[k] = str(v)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def same(a, b):
    return (a["count"] == b["count"] and a["leaf_index"] == b["leaf_index"] and a["sector"] == b["sector"]
            and np.array_equal(a["inliers"], b["inliers"]) and a["point"] == b["point"])


def solve(c, g):
    return c.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])


def read_lines(path):
    if not os.path.exists(path):
        return []
    out = []
    for line in open(path):
        f = line.split()
        assert len(f) == 5, line
        out.append((f[0], int(f[1]), int(f[2]), int(f[3]), int(f[4])))
    return out


FAMILY = {"line2d": 1, "plane3d": 2, "ray3d": 3, "pose4dof": 4, "sim2d": 5}


# every family code indexes the tuner's table, the last one included
@pytest.mark.parametrize("name", ["plane3d_small", "pose4dof_small", "sim2d_small"])
def test_autotune_cache_and_results(tmp_path, name):
    from paper_2107_11810_amd import gvote
    g = synth.config(name)
    fam = FAMILY[g["family"]]
    path = str(tmp_path / "tune.txt")
    ro = oracle.solve(oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]))
    with Env(GV_AUTOTUNE=0):
        base = gvote.Context(0)
        r0 = solve(base, g)
        base.close()
    assert r0["count"] == ro["count"] and r0["leaf_index"] == ro["leaf_index"]
    assert np.array_equal(r0["inliers"], ro["inliers"])
    with Env(GV_TUNE_MIN_BYTES=0):
        c = gvote.Context(0, autotune_cache=path)
        try:
            for i in range(64):
                _say("tune", name, i)
                assert same(solve(c, g), r0)
                kinds = {k for (_, _, f, k, _) in read_lines(path) if f == fam}
                if kinds == {0, 1, 2}:
                    break
        finally:
            c.close()
    lines = read_lines(path)
    mine = [l for l in lines if l[2] == fam]
    assert {l[3] for l in mine} == {0, 1, 2}, lines
    for arch, ncu, f, k, v in lines:
        assert ncu > 0 and f in FAMILY.values() and k in (0, 1, 2)
        assert v in (TILE_LOGS if k == 2 else CANDIDATES)
    before = open(path).read()
    # choices read back: no more tuning samples, same results, file unchanged
    with Env(GV_TUNE_MIN_BYTES=0):
        c2 = gvote.Context(0, autotune_cache=path)
        try:
            assert same(solve(c2, g), r0)
        finally:
            c2.close()
    assert open(path).read() == before


@pytest.mark.parametrize("grid", [1, 2, 32, 64])
@pytest.mark.parametrize("name", ["line2d_small", "plane3d_small", "ray3d_small", "pose4dof_small", "sim2d_small"])
def test_fixed_grids_same_result(name, grid):
    from paper_2107_11810_amd import gvote
    g = synth.config(name)
    _say("grid", name, grid)
    ro = oracle.solve(oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]))
    with Env(GV_GRID_COUNT=grid, GV_GRID_COMPACT=grid):
        c = gvote.Context(0)
        try:
            r = solve(c, g)
        finally:
            c.close()
    assert r["count"] == ro["count"] and r["leaf_index"] == ro["leaf_index"] and r["sector"] == ro["sector"]
    assert np.array_equal(r["inliers"], ro["inliers"])
    d = 4 if g["family"] == "pose4dof" else len(g["lo"])
    for j in range(d):
        assert r["point"][j] == ro["point"][j]


@pytest.mark.parametrize("tile", [256, 512])
@pytest.mark.parametrize("name", ["line2d_small", "plane3d_small", "ray3d_small", "pose4dof_small", "sim2d_small",
                                  "pose5dof_tiny"])
def test_fixed_tiles_same_result(name, tile):
    """Every batch cut into items of `tile` entries (instead of 1024, or the
    5-DoF family's smaller items for small batches) gives the oracle's
    result."""
    from paper_2107_11810_amd import gvote
    g = synth.config(name)
    _say("tile", name, tile)
    ro = oracle.solve(oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]))
    with Env(GV_ITEM_ENTRIES=tile):
        c = gvote.Context(0)
        try:
            r = solve(c, g)
        finally:
            c.close()
    assert r["count"] == ro["count"] and r["leaf_index"] == ro["leaf_index"] and r["sector"] == ro["sector"]
    assert np.array_equal(r["inliers"], ro["inliers"])
