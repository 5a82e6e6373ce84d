"""ctypes binding of libgvote.so (include/gvote.h).

Argument marshalling only: every step of the voting path runs in the HIP
library.  Columns may be numpy arrays (host) or torch CUDA/HIP tensors
(device pointers, borrowed for the duration of the call).  If the library is
not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgvote.so")

LINE2D, PLANE3D, RAY3D, POSE4DOF, SIM2D, POSE5DOF = 1, 2, 3, 4, 5, 6
FAMILIES = {"line2d": LINE2D, "plane3d": PLANE3D, "ray3d": RAY3D, "pose4dof": POSE4DOF, "sim2d": SIM2D,
            "pose5dof": POSE5DOF}
NCOLS = {LINE2D: 2, PLANE3D: 3, RAY3D: 6, POSE4DOF: 5, SIM2D: 4, POSE5DOF: 5}
AXES = 5  # GV_AXES: per-axis arrays of the ABI
FP64_PLAIN, FP32_FILTER = 0, 1

STATUS = {0: "GV_OK", -1: "GV_EINVAL", -2: "GV_ENOMEM", -3: "GV_ETOOBIG", -4: "GV_EBUFSZ",
          -5: "GV_EAGAIN", -6: "GV_ETIMEDOUT", -7: "GV_ECANCELED", -8: "GV_EDEVICE", -9: "GV_ERANGE"}

EXPORTS = ["gv_create", "gv_destroy", "gv_solve", "gv_solve_noalloc", "gv_report", "gv_parametrize", "gv_incidence",
           "gv_refine", "gv_submit",
           "gv_poll", "gv_cancel",
           "gv_status_str", "gv_last_error"]


class CtxConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("mem_budget_bytes", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("autotune_cache", ctypes.c_char_p),
                ("kernel_timing", ctypes.c_int)]


class Problem(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("n", ctypes.c_int64), ("col", ctypes.c_void_p * 6),
                ("cols_on_device", ctypes.c_int), ("lo", ctypes.c_double * AXES), ("hi", ctypes.c_double * AXES),
                ("eps", ctypes.c_double * AXES), ("canon_c", ctypes.c_double), ("precision", ctypes.c_int),
                ("group", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("tests", ctypes.c_uint64), ("fp64_rechecks", ctypes.c_uint64),
                ("cells_expanded", ctypes.c_uint64), ("cells_pruned", ctypes.c_uint64),
                ("groups_merged", ctypes.c_uint64), ("levels", ctypes.c_uint32),
                ("ms_total", ctypes.c_double), ("ms_kernels", ctypes.c_double),
                ("test_ms", ctypes.c_double), ("compact_ms", ctypes.c_double),
                ("test_launches", ctypes.c_uint64), ("compact_launches", ctypes.c_uint64),
                ("test_bytes", ctypes.c_uint64), ("compact_bytes", ctypes.c_uint64),
                ("ms_queued", ctypes.c_double), ("compact_write_bytes", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("point", ctypes.c_double * AXES), ("count", ctypes.c_uint64), ("leaf_index", ctypes.c_uint64),
                ("sector", ctypes.c_int32), ("leaf_coords", ctypes.c_int32 * AXES),
                ("inliers", ctypes.POINTER(ctypes.c_int64)), ("inliers_cap", ctypes.c_uint64),
                ("n_inliers", ctypes.c_uint64), ("bound", ctypes.c_double * AXES), ("stats", Stats)]


class Refined(ctypes.Structure):
    _fields_ = [("pose", ctypes.c_double * AXES), ("rms0", ctypes.c_double), ("rms", ctypes.c_double),
                ("verified", ctypes.POINTER(ctypes.c_int64)), ("verified_cap", ctypes.c_uint64),
                ("n_verified", ctypes.c_uint64)]


class GvError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libgvote.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2107_11810_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.gv_create.argtypes = [P(ctypes.c_void_p), P(CtxConfig)]
        L.gv_destroy.argtypes = [ctypes.c_void_p]
        L.gv_solve.argtypes = [ctypes.c_void_p, P(Problem), P(Result)]
        L.gv_solve_noalloc.argtypes = [ctypes.c_void_p, P(Problem), P(Result)]
        L.gv_report.argtypes = [ctypes.c_void_p, P(Problem), ctypes.c_uint64, P(ctypes.c_uint64), P(ctypes.c_uint32),
                                ctypes.c_uint64, P(ctypes.c_uint64), P(Stats)]
        L.gv_parametrize.argtypes = [ctypes.c_void_p, P(Problem), P(ctypes.c_double), P(ctypes.c_double),
                                     P(ctypes.c_int32)]
        L.gv_incidence.argtypes = [ctypes.c_void_p, P(Problem), ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32),
                                   P(ctypes.c_uint32), P(Stats)]
        L.gv_refine.argtypes = [ctypes.c_void_p, P(Problem), ctypes.c_uint64, P(ctypes.c_int64), ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P(Refined)]
        L.gv_submit.argtypes = [ctypes.c_void_p, P(Problem), P(ctypes.c_uint64)]
        L.gv_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(Result), ctypes.c_int]
        L.gv_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.gv_status_str.argtypes = [ctypes.c_int]
        L.gv_status_str.restype = ctypes.c_char_p
        L.gv_last_error.argtypes = [ctypes.c_void_p]
        L.gv_last_error.restype = ctypes.c_char_p
        for name in ("gv_create", "gv_destroy", "gv_solve", "gv_solve_noalloc", "gv_report", "gv_parametrize",
                     "gv_incidence", "gv_refine",
                     "gv_submit", "gv_poll", "gv_cancel"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _col_ptr(c, on_device):
    if on_device:
        return ctypes.c_void_p(int(c.data_ptr()))
    return ctypes.c_void_p(c.ctypes.data)


def make_problem(family, cols, lo, hi, eps, canon_c=0.0, precision=FP32_FILTER, group=0):
    """Fill a gv_problem from numpy arrays or device tensors (kept alive by
    the returned tuple)."""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    on_dev = bool(cols) and hasattr(cols[0], "data_ptr") and getattr(cols[0], "is_cuda", False)
    keep = []
    p = Problem()
    p.family = fam
    if on_dev:
        cs = list(cols)  # float64, contiguous device vectors
        p.n = int(cs[0].numel()) if cs else 0
    else:
        cs = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in cols]
        p.n = int(cs[0].shape[0]) if cs else 0
    if len(cs) != NCOLS[fam]:
        raise ValueError(f"family {fam} needs {NCOLS[fam]} columns")
    for k, c in enumerate(cs):
        p.col[k] = _col_ptr(c, on_dev)
        keep.append(c)
    p.cols_on_device = 1 if on_dev else 0
    for j in range(AXES):
        p.lo[j] = float(lo[j]) if j < len(lo) else 0.0
        p.hi[j] = float(hi[j]) if j < len(hi) else 0.0
        p.eps[j] = float(eps[j]) if j < len(eps) else 0.0
    p.canon_c = float(canon_c)
    p.precision = int(precision)
    p.group = int(group)
    return p, keep


class Context:
    def __init__(self, device=0, mem_budget_bytes=0, hip_stream=None, kernel_timing=False, autotune_cache=None):
        self._h = ctypes.c_void_p()
        cfg = CtxConfig()
        cfg.device = device
        cfg.mem_budget_bytes = mem_budget_bytes
        cfg.hip_stream = hip_stream
        self._tune_path = None if autotune_cache is None else os.fsencode(autotune_cache)
        cfg.autotune_cache = self._tune_path
        cfg.kernel_timing = 1 if kernel_timing else 0
        st = lib().gv_create(ctypes.byref(self._h), ctypes.byref(cfg))
        if st != 0:
            raise GvError(st, "gv_create")

    def close(self):
        if self._h:
            lib().gv_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib().gv_last_error(self._h).decode()

    def solve(self, family, cols, lo, hi, eps, canon_c=0.0, precision=FP32_FILTER, cap=None, group=0,
              noalloc=False):
        """gv_solve (or gv_solve_noalloc: no allocation, fixed scratch)."""
        p, keep = make_problem(family, cols, lo, hi, eps, canon_c, precision, group)
        cap = p.n if cap is None else cap
        buf = np.zeros(max(1, cap), dtype=np.int64)
        r = Result()
        r.inliers = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        r.inliers_cap = cap
        fn = lib().gv_solve_noalloc if noalloc else lib().gv_solve
        st = fn(self._h, ctypes.byref(p), ctypes.byref(r))
        if st != 0:
            raise GvError(st, self.last_error())
        s = r.stats
        return {
            "count": int(r.count), "leaf_index": int(r.leaf_index), "sector": int(r.sector),
            "leaf_coords": list(r.leaf_coords), "point": list(r.point), "n_inliers": int(r.n_inliers),
            "inliers": buf[: r.n_inliers].copy(), "bound": list(r.bound),
            "stats": {"tests": s.tests, "fp64_rechecks": s.fp64_rechecks, "cells_expanded": s.cells_expanded,
                      "cells_pruned": s.cells_pruned, "groups_merged": s.groups_merged, "levels": s.levels,
                      "ms_total": s.ms_total, "ms_kernels": s.ms_kernels,
                      "test_ms": s.test_ms, "compact_ms": s.compact_ms, "test_launches": s.test_launches,
                      "compact_launches": s.compact_launches, "test_bytes": s.test_bytes,
                      "compact_bytes": s.compact_bytes, "compact_write_bytes": s.compact_write_bytes},
        }

    def report(self, family, cols, lo, hi, eps, tau, cap=1 << 20, canon_c=0.0, precision=FP32_FILTER, group=0):
        """Every leaf whose count reaches tau (gv_report): (leaf indices,
        counts, stats), ascending leaf index."""
        p, keep = make_problem(family, cols, lo, hi, eps, canon_c, precision, group)
        idx = np.zeros(max(1, cap), dtype=np.uint64)
        cnt = np.zeros(max(1, cap), dtype=np.uint32)
        n = ctypes.c_uint64(0)
        st_out = Stats()
        st = lib().gv_report(self._h, ctypes.byref(p), int(tau), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(cap), ctypes.byref(n),
                             ctypes.byref(st_out))
        if st != 0:
            raise GvError(st, self.last_error())
        return idx[: n.value].copy(), cnt[: n.value].copy(), {"tests": st_out.tests, "ms_total": st_out.ms_total}

    def incidence(self, family, cols, lo, hi, eps, level, sector, coords, canon_c=0.0, precision=FP32_FILTER):
        """Pass masks of every surface against the children of one cell
        (gv_incidence); returns (masks, tests, fp64 rechecks)."""
        p, keep = make_problem(family, cols, lo, hi, eps, canon_c, precision)
        cc = (ctypes.c_int32 * AXES)(*[int(c) for c in list(coords) + [0] * (AXES - len(coords))])
        masks = np.zeros(max(1, p.n), dtype=np.uint32)
        st_out = Stats()
        st = lib().gv_incidence(self._h, ctypes.byref(p), int(level), int(sector), cc,
                                masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st_out))
        if st != 0:
            raise GvError(st, self.last_error())
        return masks[: p.n], int(st_out.tests), int(st_out.fp64_rechecks)

    def refine(self, family, cols, lo, hi, eps, leaf_index, idx, tau0, tau, rounds=2, iters=10):
        """Angular verification and Gauss-Newton refinement after the vote
        (gv_refine): returns {pose, verified, rms, rms0}."""
        p, keep = make_problem(family, cols, lo, hi, eps)
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        buf = np.zeros(max(1, idx.size), dtype=np.int64)
        out = Refined()
        out.verified = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        out.verified_cap = idx.size
        st = lib().gv_refine(self._h, ctypes.byref(p), int(leaf_index),
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size, float(tau0), float(tau),
                             int(rounds), int(iters), ctypes.byref(out))
        if st != 0:
            raise GvError(st, self.last_error())
        return {"pose": list(out.pose), "verified": buf[: out.n_verified].copy(), "rms": out.rms,
                "rms0": out.rms0}

    def parametrize(self, family, cols, lo, hi, eps):
        p, keep = make_problem(family, cols, lo, hi, eps)
        n = p.n
        t = np.zeros((max(n, 1), 4))
        f = np.zeros((max(n, 1), 2))
        tag = np.zeros(max(n, 1), dtype=np.int32)
        st = lib().gv_parametrize(self._h, ctypes.byref(p), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  tag.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if st != 0:
            raise GvError(st, self.last_error())
        return t[:n], f[:n], tag[:n]


# ---------------------------------------------------------------------------
# Device buffers through the same HIP runtime the library links (one runtime
# per process): inputs resident in HBM before a timed solve.
# ---------------------------------------------------------------------------
_hip = None


def hip():
    global _hip
    if _hip is None:
        lib()  # the library pulls in its HIP runtime first
        H = ctypes.CDLL("libamdhip64.so.7")
        H.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        H.hipFree.argtypes = [ctypes.c_void_p]
        H.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        H.hipDeviceSynchronize.argtypes = []
        for f in (H.hipMalloc, H.hipFree, H.hipMemcpy, H.hipDeviceSynchronize):
            f.restype = ctypes.c_int
        _hip = H
    return _hip


class DeviceArray:
    """A float64 vector in device memory (hipMalloc), filled from numpy."""

    def __init__(self, a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self.n = int(a.shape[0])
        self.ptr = ctypes.c_void_p()
        st = hip().hipMalloc(ctypes.byref(self.ptr), max(8, a.nbytes))
        if st != 0:
            raise GvError(-2, f"hipMalloc failed ({st})")
        if a.nbytes:
            st = hip().hipMemcpy(self.ptr, ctypes.c_void_p(a.ctypes.data), a.nbytes, 1)  # host -> device
            if st != 0:
                raise GvError(-8, f"hipMemcpy failed ({st})")
        self.is_cuda = True

    def data_ptr(self):
        return self.ptr.value

    def numel(self):
        return self.n

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def to_device(cols):
    return [DeviceArray(c) for c in cols]


# ---------------------------------------------------------------------------
# Continuous batching
# ---------------------------------------------------------------------------
def _result_dict(r, buf):
    s = r.stats
    return {"count": int(r.count), "leaf_index": int(r.leaf_index), "sector": int(r.sector),
            "leaf_coords": list(r.leaf_coords), "point": list(r.point), "n_inliers": int(r.n_inliers),
            "inliers": buf[: r.n_inliers].copy(), "bound": list(r.bound),
            "stats": {"tests": s.tests, "fp64_rechecks": s.fp64_rechecks, "ms_total": s.ms_total,
                      "ms_queued": s.ms_queued}}


def submit(ctx, family, cols, lo, hi, eps, canon_c=0.0, precision=FP32_FILTER, group=0):
    """Enqueue a problem; returns its ticket (host columns are copied)."""
    p, keep = make_problem(family, cols, lo, hi, eps, canon_c, precision, group)
    t = ctypes.c_uint64(0)
    st = lib().gv_submit(ctx._h, ctypes.byref(p), ctypes.byref(t))
    if st != 0:
        raise GvError(st, ctx.last_error())
    return t.value


def poll(ctx, ticket, cap, timeout_ms=-1):
    """Wait for a ticket; returns (status, result dict or None)."""
    buf = np.zeros(max(1, cap), dtype=np.int64)
    r = Result()
    r.inliers = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    r.inliers_cap = cap
    st = lib().gv_poll(ctx._h, ctypes.c_uint64(ticket), ctypes.byref(r), int(timeout_ms))
    if st != 0:
        return st, ({"n_inliers": int(r.n_inliers)} if st == -4 else None)
    return 0, _result_dict(r, buf)


def cancel(ctx, ticket):
    return lib().gv_cancel(ctx._h, ctypes.c_uint64(ticket))
