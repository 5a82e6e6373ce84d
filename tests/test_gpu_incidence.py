"""Device parity of single steps and modes, through the C ABI:

  * the incidence test alone (gv_incidence): pass masks of every surface,
    canonized along the path to a cell, against that cell's children, for
    every family, in both precisions, bit-equal to the oracle;
  * the binary32 filter at its thresholds: 4-DoF pose surfaces placed exactly
    on, and a few lattice steps or a few binary32 rounding units from, each
    sign decision of the test (z low and high ends for either sign of eta,
    the apex guard, and the four cross products of the kappa cone); the
    filtered masks equal the binary64 ones and the oracle's, and the filter
    does leave decisions to binary64 there;
  * exact mode (canon_c = +inf), the plain definition, against the oracle's;
  * the certified bound: every reported inlier lies within it, by direct
    binary64 evaluation of its observation against the returned leaf;
  * the deepest lattices the linear families accept, with ragged item tails.
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle
import test_oracle_bounds as TB
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


def _dims(g):
    return 4 if g["family"] == "pose4dof" else len(g["lo"])


def check_same(g, r_gpu, r_or):
    assert r_gpu["count"] == r_or["count"], (r_gpu["count"], r_or["count"])
    assert r_gpu["leaf_index"] == r_or["leaf_index"]
    assert r_gpu["sector"] == r_or["sector"]
    assert np.array_equal(r_gpu["inliers"], r_or["inliers"])
    d = _dims(g)
    assert r_gpu["leaf_coords"][:d] == r_or["leaf_coords"][:d]
    for j in range(d):
        assert r_gpu["point"][j] == r_or["point"][j]


# ----------------------------------------------------------------------------
# Incidence test alone
# ----------------------------------------------------------------------------
def _random_cells(g, rng, k):
    E, epsn, L, Ls, B = TB.geometry(g)
    out = []
    for _ in range(k):
        m = int(rng.integers(0, Ls))
        cc = [int(rng.integers(0, 2 ** min(m, L[j]))) for j in range(len(L))]
        sec = int(rng.integers(0, 4)) if g["family"] == "pose4dof" else 0
        out.append((m, sec, cc))
    return out


@pytest.mark.parametrize("name", ["line2d_small", "plane3d_small", "ray3d_small", "pose4dof_small", "line2d_tiny",
                                  "ray3d_tiny", "pose4dof_small_flat", "sim2d_tiny", "sim2d_small"])
@pytest.mark.parametrize("exact", [False, True])
def test_incidence_masks_equal_the_oracle(ctx, name, exact):
    g = synth.config(name)
    c = math.inf if exact else 0.0
    pr = OP(g, canon_c=c)
    rng = np.random.default_rng(41)
    for m, sec, cc in _random_cells(g, rng, 6):
        _say("incidence", name, "exact" if exact else "", m, sec, cc)
        mo = oracle.cell_masks(pr, m, sec, cc)
        for prec in (0, 1):
            mg, tests, rech = ctx.incidence(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], m, sec, cc,
                                            canon_c=c, precision=prec)
            assert np.array_equal(mg, mo), (m, sec, cc, prec, int(np.sum(mg != mo)))
            assert tests > 0


# ----------------------------------------------------------------------------
# Binary32 filter at its thresholds (4-DoF pose)
# ----------------------------------------------------------------------------
BOX = dict(lo=[0.0, 0.0, 0.0, 0.0], hi=[200.0, 200.0, 200.0, 2 * math.pi], eps=[4.0, 4.0, 4.0, math.radians(2.0)])
CELL = (3, 0, [1, 1, 3, 5])  # level, sector, coordinates: children at level 4 with kappa in [0.25, 0.5]


def _anchors():
    """Two matches that fix the data bounds of the pose lattice: |eta'| = 1
    and an apex in a corner of the unit square (farthest reach sqrt(2))."""
    W = np.array([[0.0, 0.0, 0.5], [1.0, 1.0, 0.5]])
    return W, np.array([0.0, 0.0]), np.array([1.0, -1.0])


def _pose_problem(W, xi, eta):
    """Observation columns from normalized lattice values (lo = 0, E = 200 on
    every metric axis, so eta' = eta)."""
    aW, axi, aeta = _anchors()
    W = np.concatenate([aW, W])
    xi = np.concatenate([axi, xi])
    eta = np.concatenate([aeta, eta])
    cols = [W[:, 0] * 200.0, W[:, 1] * 200.0, W[:, 2] * 200.0, xi, eta]
    return dict(family="pose4dof", cols=cols, **BOX)


def _lattice():
    k = oracle.constants(OP(_pose_problem(np.zeros((0, 3)), np.zeros(0), np.zeros(0))))
    sW, sW3, sXi, sEta = k["steps"]
    return dict(sW=sW, sW3=sW3, sXi=sXi, sEta=sEta, padz=k["pad0"][0], padk=k["pad0"][1], Rg=k["Rg"], L=k["L"])


def _child_boxes(lat):
    m, sec, cc = CELL
    h = 2.0 ** -(m + 1)
    box = {}
    for b in (0, 1):
        box[("X", b)] = ((2 * cc[0] + b) * h, (2 * cc[0] + b + 1) * h)
        box[("Y", b)] = ((2 * cc[1] + b) * h, (2 * cc[1] + b + 1) * h)
        box[("Z", b)] = ((2 * cc[2] + b) * h - lat["padz"], (2 * cc[2] + b + 1) * h + lat["padz"])
        klo = 2 * (2 * cc[3] + b) * h - 1
        box[("K", b)] = (klo - lat["padk"], klo + 2 * h + lat["padk"])
    return box, h


def _q(x, s):
    """x on the lattice of step s (exactly)."""
    v = x / s
    assert v == round(v), (x, s)
    return x


def _adversarial(kind, rng):
    """Matches (W1, W2, W3, xi, eta') placed at one sign decision of the test
    against the children of CELL, on the root lattice."""
    lat = _lattice()
    sW, sW3, sXi, sEta = lat["sW"], lat["sW3"], lat["sXi"], lat["sEta"]
    box, h = _child_boxes(lat)
    rows = []
    # a leg length of 3 q, 4 q (q a power of two in units of sW) with the
    # hypotenuse 5 q: exact squared distances, and (3q + 4)^2 + (4q - 3)^2 =
    # (5q)^2 + 25: the same distance plus 25 sW^2, a relative change far
    # below the binary32 rounding of the squares
    q = 2.0 ** math.ceil(math.log2(h / (3 * sW)))
    for bx in (0, 1):
        for by in (0, 1):
            Xlo, Xhi = box[("X", bx)]
            Ylo, Yhi = box[("Y", by)]
            for bz in (0, 1):
                ZL, ZH = box[("Z", bz)]
                if kind in ("zlo", "zhi"):
                    for sgn in (1.0, -1.0):
                        for dxy in ((0, 0), (4, -3), (-3, 4)):
                            # rmax: apex beyond the box's upper-right corner, the far corner
                            # (Xlo, Ylo) at legs (3q, 4q); rmin: the near corner (Xhi, Yhi)
                            far = kind == "zlo"
                            d1, d2 = 3 * q * sW + dxy[0] * sW, 4 * q * sW + dxy[1] * sW
                            W1 = (Xlo if far else Xhi) + d1
                            W2 = (Ylo if far else Yhi) + d2
                            r = 5 * q * sW
                            eta = _q(0.5, sEta)
                            T = _q(eta * r, sW3)  # eta' r on the z lattice: an exact tie
                            # z-lo: eta' r_max = W3 - ZH (eta > 0) or ZL - W3 (eta < 0)
                            # z-hi: eta' r_min = W3 - ZL (eta > 0) or ZH - W3 (eta < 0)
                            for dz in (-1, 0, 1):
                                if sgn > 0:
                                    W3 = (ZH + T if far else ZL + T) + dz * sW3
                                else:
                                    W3 = (ZL - T if far else ZH - T) + dz * sW3
                                xi = _q(sXi * int(rng.integers(-64, 65)), sXi)
                                rows.append((W1, W2, W3, xi, sgn * eta))
            if kind == "guard":
                for d in (-2, -1, 0, 1, 2):
                    W1 = Xhi + lat["Rg"] + d * sW
                    W2 = (Ylo + Yhi) / 2
                    for bz in (0, 1):
                        ZL, ZH = box[("Z", bz)]
                        rows.append((W1, W2, (ZL + ZH) / 2, 0.0, 0.0))
            if kind in ("c1", "c2", "c3", "c4"):
                # V (sector 0) in the open first quadrant: start corner a = (x1, y0),
                # end corner b = (x0, y1); kappa = v2/v1 when xi = 0
                for bk in (0, 1):
                    Llo, Lhi = box[("K", bk)]
                    L = Llo if kind in ("c1", "c3") else Lhi
                    for j in (11, 13, 17):
                        x0 = j * (sW / sXi)  # L x0 and L (x0 + h) stay on the xy lattice
                        for d in (-2, -1, 0, 1, 2):
                            W1 = Xhi + x0
                            if kind in ("c1", "c2"):   # a on the edge: y0 = L x1
                                W2 = Yhi + L * (x0 + h)
                            else:                      # b on the edge: y1 = L x0
                                W2 = Ylo + L * x0
                            W2 = _q(W2, sW) + d * sW
                            if W1 > 1.0 or W2 > 1.0 or W2 - Yhi <= 0:
                                continue
                            for bz in (0, 1):
                                ZL, ZH = box[("Z", bz)]
                                rows.append((W1, W2, (ZL + ZH) / 2, 0.0, 0.0))
                                # the same edge with a general xi: the nearest lattice point
                                xi = sXi * int(rng.integers(-400, 401))
                                k = Fraction(L)
                                xf = Fraction(xi)
                                num, den = k + xf, 1 - k * xf  # direction (den, num) has kappa = L
                                if kind in ("c1", "c2"):
                                    y = float(Fraction(x0 + h) * num / den)
                                    W2b = Yhi + y
                                else:
                                    y = float(Fraction(x0) * num / den)
                                    W2b = Ylo + y
                                W2b = round(W2b / sW) * sW + d * sW
                                if 0.0 < W2b - Yhi and W2b <= 1.0:
                                    rows.append((W1, W2b, (ZL + ZH) / 2, xi, 0.0))
    A = np.array(rows, dtype=np.float64)
    for col, s in zip(range(5), (sW, sW, sW3, sXi, sEta)):
        assert np.all(A[:, col] / s == np.round(A[:, col] / s)), kind
    assert np.all(np.abs(A[:, 4]) <= 1.0) and np.all((A[:, :2] >= 0) & (A[:, :2] <= 1))
    return A, lat


@pytest.mark.parametrize("kind", ["zlo", "zhi", "guard", "c1", "c2", "c3", "c4"])
def test_binary32_filter_at_the_thresholds(ctx, kind):
    rng = np.random.default_rng(7)
    A, lat = _adversarial(kind, rng)
    g = _pose_problem(A[:, :3], A[:, 3], A[:, 4])
    pr = OP(g)
    # the anchors fix the lattice; the surfaces are exactly where they were placed
    assert oracle.constants(pr)["steps"] == oracle.constants(OP(_pose_problem(np.zeros((0, 3)), np.zeros(0),
                                                                               np.zeros(0))))["steps"]
    t, f, _ = oracle.parametrize(pr, root_canon=True)
    assert np.array_equal(t[2:, 0], A[:, 0]) and np.array_equal(t[2:, 1], A[:, 1])
    assert np.array_equal(f[2:, 0], A[:, 2]) and np.array_equal(t[2:, 2], A[:, 3])
    assert np.array_equal(t[2:, 3], A[:, 4])
    m, sec, cc = CELL
    _say("filter", kind, len(A), "surfaces")
    mo = oracle.cell_masks(pr, m, sec, cc)
    m64, _, r64 = ctx.incidence(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], m, sec, cc, precision=0)
    m32, tests, r32 = ctx.incidence(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], m, sec, cc, precision=1)
    _say("  rechecks", r32, "of", tests, "tests; passes", int(np.sum([bin(int(x)).count("1") for x in m32])))
    assert r64 == 0
    assert np.array_equal(m64, mo)
    assert np.array_equal(m32, mo)
    assert r32 > 0
    # decisions on both sides of every threshold were exercised
    assert np.any(mo != 0) and np.any(mo != 0xFFFF)
    # the whole search on these surfaces: both precisions give the oracle's result
    ro = oracle.solve(pr)
    for prec in (0, 1):
        rg = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], precision=prec)
        check_same(g, rg, ro)


# ----------------------------------------------------------------------------
# Exact mode
# ----------------------------------------------------------------------------
FAMS = ["line2d", "plane3d", "ray3d", "pose4dof", "sim2d"]


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_exact_mode_tiny(ctx, fam, seed):
    g = synth.config(fam + "_tiny", seed=seed)
    _say("exact tiny", fam, seed)
    ro = oracle.solve(OP(g, canon_c=math.inf))
    for prec in (0, 1):
        rg = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf, precision=prec)
        check_same(g, rg, ro)


@pytest.mark.parametrize("fam", FAMS)
def test_exact_mode_small(ctx, fam):
    g = synth.config(fam + "_small")
    _say("exact small", fam)
    ro = oracle.solve(OP(g, canon_c=math.inf))
    rg = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf)
    check_same(g, rg, ro)
    # forced grouping in every cell changes nothing
    rg2 = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf, group=1)
    check_same(g, rg2, ro)


def test_exact_mode_equals_plain_definition(ctx):
    """On the tiny problems the oracle's exact mode is pinned to a brute force
    of the plain definition; the device matches it bit for bit."""
    import test_oracle_pins as TP
    for name, seed in [("line2d_tiny", 1), ("plane3d_tiny", 3), ("ray3d_tiny", 2)]:
        g = synth.config(name, seed=seed)
        votes, idx, bc, bi, *_ = TP._exact_bruteforce(g, OP(g, canon_c=math.inf))
        rg = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf)
        assert (rg["count"], rg["leaf_index"]) == (bc, bi)


# ----------------------------------------------------------------------------
# Certified bound
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["line2d_small", "plane3d_small", "ray3d_small", "pose4dof_small", "line2d_10k",
                                  "pose4dof_small_flat", "pose4dof_tiny", "sim2d_small"])
@pytest.mark.parametrize("exact", [False, True])
def test_every_inlier_within_the_reported_bound(ctx, name, exact):
    g = synth.config(name)
    _say("bound", name, exact)
    r = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], canon_c=math.inf if exact else 0.0)
    E, epsn, L, Ls, B = TB.geometry(g)
    pose = g["family"] == "pose4dof"
    d = len(L)
    lc = r["leaf_coords"][:d]
    lo = np.array(g["lo"][:d], float)
    if pose:
        lo[3] = -1.0
    h = np.array([E[j] * 2.0 ** -L[j] for j in range(d)])
    blo = (lo + np.array(lc) * h)[None, :]
    bhi = (lo + (np.array(lc) + 1) * h)[None, :]
    bound = r["bound"]
    assert all(b > 0 for b in bound[:d])
    # the point is the leaf centre: within the half side of every point of the leaf
    for j in range(3 if pose else d):
        assert abs(r["point"][j] - (blo[0, j] + bhi[0, j]) / 2) <= 1e-9 * E[j]
        assert bound[j] >= 0.5 * h[j] * (1 - 1e-12)
    if not pose:
        # dependent axes: no looser than eps + the allowance of Sec. 3.2 (eps/c)
        for i in r["inliers"]:
            for q, dist in TB._lin_distances(g, int(i), blo, bhi):
                assert dist[0] <= bound[q] * (1 + 1e-9), (i, q, float(dist[0]), bound[q])
        for q in range(d):
            if g["family"] == "ray3d" or (q >= 2 if g["family"] == "sim2d" else q == d - 1):
                assert g["eps"][q] <= bound[q] <= (2.0 * g["eps"][q] + 1e-9) * (1.0 if not exact else 1.0)
        return
    ez, ek, pzm, pkm, Rg = TB.pose_bounds(g)
    assert g["eps"][2] <= bound[2] and g["eps"][3] <= bound[3]
    sec = np.array([r["sector"]])
    far = 0
    for i in r["inliers"]:
        zdist, rmin, p0, p1 = TB._pose_parts(g, int(i), blo, bhi, sec)
        assert zdist[0] <= bound[2] * (1 + 1e-9), (i, float(zdist[0]), bound[2])
        if rmin[0] >= Rg * E[0] * (1 + 1e-9):
            kb = bound[3] * 1.02
            ok = TB._overlap_mod(p0, p1, np.arctan(blo[:, 3] - kb) - 1e-9, np.arctan(bhi[:, 3] + kb) + 1e-9)
            assert ok[0], i
            far += 1
    assert far > 0


# ----------------------------------------------------------------------------
# The deepest lattice the linear families accept, ragged tails
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [37, 100, 1000])
def test_deep_lattice_and_ragged_items(ctx, n):
    """Unit box, eps 2^-21: the free step is 2^-27 and a level-0 cell spans
    2^27 lattice steps, the largest the 32-bit lattice accepts; n not a
    multiple of the wave size leaves idle lanes in the last block of every
    item, which must pass no child."""
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 1, n)
    a, b = 0.3125, 0.40625
    y = np.where(np.arange(n) < n // 3, a * x + b, rng.uniform(0, 1, n))
    g = dict(family="line2d", cols=[x, y], lo=[0.0, 0.0], hi=[1.0, 1.0], eps=[2.0 ** -21, 2.0 ** -21])
    _say("deep lattice", n)
    ro = oracle.solve(OP(g))
    rg = ctx.solve(g["family"], g["cols"], g["lo"], g["hi"], g["eps"])
    check_same(g, rg, ro)
    assert rg["count"] >= n // 3
