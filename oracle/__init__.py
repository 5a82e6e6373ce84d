"""CPU FP64 oracle for the general-voting maximum-depth search.

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  The C source (``gv_oracle.c``) shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gv_oracle.c")
_LIB = os.path.join(_HERE, "libgv_oracle.so")

FAMILIES = {"line2d": 1, "plane3d": 2, "ray3d": 3, "pose4dof": 4, "sim2d": 5, "pose5dof": 6}
NCOLS = {1: 2, 2: 3, 3: 6, 4: 5, 5: 4, 6: 5}
POSE = (4, 6)  # the camera-posing families: four yaw sectors on top of the leaf index
MAXD = 5

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EBUFSZ", -4: "ERANGE", -5: "EBUDGET"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-pthread", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("family", ctypes.c_int),
        ("n", ctypes.c_int64),
        ("col", ctypes.POINTER(ctypes.c_double) * 6),
        ("lo", ctypes.c_double * MAXD),
        ("hi", ctypes.c_double * MAXD),
        ("eps", ctypes.c_double * MAXD),
        ("canon_c", ctypes.c_double),
        ("no_prune", ctypes.c_int),
        ("no_group", ctypes.c_int),
        ("no_dive", ctypes.c_int),
        ("test_budget", ctypes.c_uint64),
        ("threads", ctypes.c_int),
        ("has_seed", ctypes.c_int),
        ("seed_leaf", ctypes.c_uint64),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64),
        ("leaf_index", ctypes.c_uint64),
        ("key", ctypes.c_uint64),
        ("sector", ctypes.c_int32),
        ("leaf_coords", ctypes.c_int32 * MAXD),
        ("levels", ctypes.c_int32 * MAXD),
        ("lstar", ctypes.c_int32),
        ("index_bits", ctypes.c_int32),
        ("point", ctypes.c_double * MAXD),
        ("n_inliers", ctypes.c_int64),
        ("tests", ctypes.c_uint64),
        ("cells_expanded", ctypes.c_uint64),
        ("cells_pruned", ctypes.c_uint64),
        ("groups_merged", ctypes.c_uint64),
        ("seconds", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.or_solve.argtypes = [P(_Problem), P(_Result), P(ctypes.c_int64), ctypes.c_int64]
        L.or_parametrize.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int32)]
        L.or_root_canon.argtypes = L.or_parametrize.argtypes
        L.or_leaf_count.argtypes = [P(_Problem), ctypes.c_uint64, P(ctypes.c_uint64), P(ctypes.c_int64),
                                    ctypes.c_int64]
        L.or_all_leaf_counts.argtypes = [P(_Problem), P(ctypes.c_uint32), ctypes.c_uint64]
        L.or_level_counts.argtypes = [P(_Problem), ctypes.c_int, P(ctypes.c_uint32), ctypes.c_uint64]
        L.or_leaf_indicator.argtypes = [P(_Problem), ctypes.c_int64, P(ctypes.c_uint8), ctypes.c_uint64]
        L.or_report.argtypes = [P(_Problem), ctypes.c_uint64, P(ctypes.c_uint64), P(ctypes.c_uint32), ctypes.c_int64,
                                P(ctypes.c_int64), P(ctypes.c_uint64)]
        L.or_cell_masks.argtypes = [P(_Problem), ctypes.c_int, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_uint32)]
        L.or_meets.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32,
                               ctypes.c_int, ctypes.c_int32, P(ctypes.c_int32)]
        L.or_canon_at.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32,
                                  ctypes.c_int, P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double)]
        L.or_constants.argtypes = [P(_Problem), P(ctypes.c_double), ctypes.c_int]
        L.or_refine.argtypes = [P(_Problem), ctypes.c_uint64, P(ctypes.c_int64), ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_int64),
                                P(ctypes.c_double), P(ctypes.c_double)]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what}: {STATUS.get(status, status)}")
        self.status = status


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """A voting problem: observation columns (SoA), domain box, per-axis eps."""

    def __init__(self, family, cols, lo, hi, eps, canon_c=0.0, no_prune=False, no_group=False,
                 no_dive=False, test_budget=0, threads=1, seed_leaf=None):
        self.family = FAMILIES[family] if isinstance(family, str) else int(family)
        self.cols = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in cols]
        if len(self.cols) != NCOLS[self.family]:
            raise ValueError("wrong number of columns")
        self.n = int(self.cols[0].shape[0]) if self.cols else 0
        self.lo = list(lo) + [0.0] * (MAXD - len(lo))
        self.hi = list(hi) + [0.0] * (MAXD - len(hi))
        self.eps = list(eps) + [0.0] * (MAXD - len(eps))
        self.canon_c = float(canon_c)
        self.no_prune, self.no_group, self.no_dive = no_prune, no_group, no_dive
        self.test_budget = int(test_budget)
        self.threads = int(threads)
        self.seed_leaf = seed_leaf

    def _c(self):
        p = _Problem()
        p.family = self.family
        p.n = self.n
        for k, c in enumerate(self.cols):
            p.col[k] = _dptr(c)
        for j in range(MAXD):
            p.lo[j], p.hi[j], p.eps[j] = self.lo[j], self.hi[j], self.eps[j]
        p.canon_c = self.canon_c
        p.no_prune, p.no_group, p.no_dive = int(self.no_prune), int(self.no_group), int(self.no_dive)
        p.test_budget = self.test_budget
        p.threads = self.threads
        p.has_seed = 0 if self.seed_leaf is None else 1
        p.seed_leaf = 0 if self.seed_leaf is None else int(self.seed_leaf)
        return p


def solve(prob: Problem, cap: int | None = None) -> dict:
    cap = prob.n if cap is None else cap
    inl = np.zeros(max(cap, 1), dtype=np.int64)
    r = _Result()
    p = prob._c()
    st = lib().or_solve(ctypes.byref(p), ctypes.byref(r), inl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap)
    if st != 0 and not (st == -5):
        raise OracleError(st, "solve")
    out = {
        "status": st,
        "count": r.count, "leaf_index": r.leaf_index, "key": r.key, "sector": r.sector,
        "leaf_coords": list(r.leaf_coords), "levels": list(r.levels), "lstar": r.lstar,
        "index_bits": r.index_bits, "point": list(r.point), "n_inliers": r.n_inliers,
        "inliers": inl[: min(r.n_inliers, cap)].copy(),
        "tests": r.tests, "cells_expanded": r.cells_expanded, "cells_pruned": r.cells_pruned,
        "groups_merged": r.groups_merged, "seconds": r.seconds,
    }
    return out


def parametrize(prob: Problem, root_canon: bool = False):
    n = prob.n
    t = np.zeros((max(n, 1), 4))
    f = np.zeros((max(n, 1), 2))
    tag = np.zeros(max(n, 1), dtype=np.int32)
    p = prob._c()
    fn = lib().or_root_canon if root_canon else lib().or_parametrize
    st = fn(ctypes.byref(p), _dptr(t), _dptr(f), tag.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if st != 0:
        raise OracleError(st, "parametrize")
    return t[:n], f[:n], tag[:n]


def leaf_count(prob: Problem, leaf_index: int, with_inliers: bool = False):
    cnt = ctypes.c_uint64(0)
    p = prob._c()
    if with_inliers:
        inl = np.zeros(max(prob.n, 1), dtype=np.int64)
        st = lib().or_leaf_count(ctypes.byref(p), leaf_index, ctypes.byref(cnt),
                                 inl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), prob.n)
        if st != 0:
            raise OracleError(st, "leaf_count")
        return cnt.value, inl[: cnt.value].copy()
    st = lib().or_leaf_count(ctypes.byref(p), leaf_index, ctypes.byref(cnt), None, 0)
    if st != 0:
        raise OracleError(st, "leaf_count")
    return cnt.value


def all_leaf_counts(prob: Problem) -> np.ndarray:
    k = constants(prob)
    B = int(k["B"])
    out = np.zeros(1 << B, dtype=np.uint32)
    p = prob._c()
    st = lib().or_all_leaf_counts(ctypes.byref(p), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), out.size)
    if st != 0:
        raise OracleError(st, "all_leaf_counts")
    return out


def level_counts(prob: Problem, level: int) -> np.ndarray:
    """Chain counts of every cell of one level (index = [sector] || digits)."""
    k = constants(prob)
    bits = (2 if prob.family in POSE else 0) + sum(
        sum(1 for j in range(MAXD) if m < k["L"][j]) for m in range(level))
    out = np.zeros(1 << bits, dtype=np.uint32)
    p = prob._c()
    st = lib().or_level_counts(ctypes.byref(p), int(level), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               out.size)
    if st != 0:
        raise OracleError(st, "level_counts")
    return out


def leaf_indicator(prob: Problem, i: int) -> np.ndarray:
    """1 at every leaf where surface i is counted (its chain passes)."""
    k = constants(prob)
    out = np.zeros(1 << int(k["B"]), dtype=np.uint8)
    p = prob._c()
    st = lib().or_leaf_indicator(ctypes.byref(p), int(i), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                 out.size)
    if st != 0:
        raise OracleError(st, "leaf_indicator")
    return out


def report(prob: Problem, tau: int, cap: int = 1 << 20):
    """Every leaf whose count reaches tau: (leaf indices, counts), index order."""
    idx = np.zeros(max(1, cap), dtype=np.uint64)
    cnt = np.zeros(max(1, cap), dtype=np.uint32)
    n = ctypes.c_int64(0)
    tests = ctypes.c_uint64(0)
    p = prob._c()
    st = lib().or_report(ctypes.byref(p), int(tau), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                         cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap, ctypes.byref(n),
                         ctypes.byref(tests))
    if st != 0:
        raise OracleError(st, "report")
    return idx[: n.value].copy(), cnt[: n.value].copy()


def cell_masks(prob: Problem, level: int, sector: int, coords) -> np.ndarray:
    """Pass masks (bit = child digit) of every surface, canonized along the
    path to the cell, against the children of that cell."""
    cc = np.ascontiguousarray(np.asarray(list(coords) + [0] * (MAXD - len(coords)), dtype=np.int32))
    out = np.zeros(max(1, prob.n), dtype=np.uint32)
    p = prob._c()
    st = lib().or_cell_masks(ctypes.byref(p), int(level), int(sector), cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if st != 0:
        raise OracleError(st, "cell_masks")
    return out[: prob.n]


def meets(prob: Problem, t, f, tag, level, sector, coords) -> bool:
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(4))
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(2))
    cc = np.ascontiguousarray(np.asarray(list(coords) + [0] * (MAXD - len(coords)), dtype=np.int32))
    p = prob._c()
    st = lib().or_meets(ctypes.byref(p), _dptr(t), _dptr(f), int(tag), int(level), int(sector),
                        cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if st < 0:
        raise OracleError(st, "meets")
    return bool(st)


def canon_at(prob: Problem, t, f, tag, level, coords):
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(4))
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(2))
    cc = np.ascontiguousarray(np.asarray(list(coords) + [0] * (MAXD - len(coords)), dtype=np.int32))
    to = np.zeros(4)
    fo = np.zeros(2)
    p = prob._c()
    st = lib().or_canon_at(ctypes.byref(p), _dptr(t), _dptr(f), int(tag), int(level),
                           cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(to), _dptr(fo))
    if st != 0:
        raise OracleError(st, "canon_at")
    return to, fo


def constants(prob: Problem) -> dict:
    out = np.zeros(27)
    p = prob._c()
    st = lib().or_constants(ctypes.byref(p), _dptr(out), 27)
    if st != 0:
        raise OracleError(st, "constants")
    d = {"Lstar": int(out[0]), "B": int(out[1]), "L": [int(x) for x in out[2:6]] + [int(out[24])],
         "steps": list(out[6:10]), "pad0": list(out[10:14]), "padlast": list(out[14:18]),
         "Rg": out[18], "epsn": list(out[19:23]) + [out[25]], "exact": bool(out[23]), "Fb": out[26]}
    return d


def refine(prob: Problem, leaf_index: int, idx, tau0: float, tau: float, rounds: int = 2, iters: int = 10) -> dict:
    """Angular verification of the vote's inliers idx (tau0 at the centre of
    leaf_index, tau after each round) and Gauss-Newton refinement of the pose
    (pose families)."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    pose = np.zeros(MAXD)
    ver = np.zeros(max(1, idx.size), dtype=np.int64)
    nv = ctypes.c_int64(0)
    rms = ctypes.c_double(0.0)
    rms0 = ctypes.c_double(0.0)
    p = prob._c()
    st = lib().or_refine(ctypes.byref(p), int(leaf_index), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         idx.size, float(tau0), float(tau), int(rounds), int(iters), _dptr(pose),
                         ver.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(nv), ctypes.byref(rms),
                         ctypes.byref(rms0))
    if st != 0:
        raise OracleError(st, "refine")
    return {"pose": list(pose), "verified": ver[: nv.value].copy(), "rms": rms.value, "rms0": rms0.value}


def leaf_index_of(levels, coords, sector=None) -> int:
    """Leaf index from per-axis leaf coordinates: digits of levels 0..L*-1,
    each holding the split axes' bits in axis order, MSB first; the pose
    families' sector goes on top."""
    d = len(levels)
    lstar = max(levels)
    idx = 0 if sector is None else int(sector)
    for m in range(lstar):
        for j in range(d):
            if m < levels[j]:
                bit = (int(coords[j]) >> (levels[j] - 1 - m)) & 1
                idx = (idx << 1) | bit
    return idx


def pose_point_yaw(sector: int, kappa: float) -> float:
    y = sector * (math.pi / 2.0) + math.atan(kappa)
    if y < 0:
        y += 2 * math.pi
    if y >= 2 * math.pi:
        y -= 2 * math.pi
    return y
