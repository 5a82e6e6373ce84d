"""Pins of the oracle's 5-DoF camera-posing family (Sec. 4.2.1: known gravity
direction, unknown focal length; axes x, y, z, kappa, f) against what the
surface equations and the mathematics fix, computed here from the problem's
box, eps and canon constant alone (never from the oracle's own constants):

  * closed form: a noise-free match of a known pose (x*, y*, z*, theta*, f*)
    gives a surface through it, z* = w3 - eta f* r and kappa = tan(theta* -
    s pi/2) with s the sector of theta*;
  * the 4-DoF family is the case f = 1: a 5-DoF problem whose f interval is
    [1, 1 + 2^-40] gives the 4-DoF problem's leaf counts and result;
  * predicate: sound (a cell that holds a point within eps of the surface
    on each dependent axis passes) and tight (a passing cell holds a point
    within the pad bound plus the sampling resolution), the z range over a
    cell taken in closed form from its range of horizontal distances and of
    f, kappa compared as an angle on a dense (x, y, f) grid;
  * the root lattice moves z and kappa by at most eps'/2 anywhere on the box;
  * search: the argmax of every leaf's chain count (tiny problems), the same
    without pruning, grouping or dive and with a thread pool;
  * (LOW) and (UP) at every leaf of tiny problems, from the match itself;
  * counts shrink down the tree; the returned point is the centre of the
    returned leaf and lies near the planted truth; the leaf levels of the
    benchmark workload.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth
from test_oracle_bounds import _angle_span, _overlap_mod, _rot, decode_leaf, leaf_grid, levels_of

ELL = 4  # essential parameters w1, w2, xi, eta


def P(g, **kw):
    return oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], **kw)


def geometry5(g):
    """Extents (kappa spans [-1, 1]), leaf levels, L*, index bits."""
    E = [g["hi"][j] - g["lo"][j] for j in range(3)] + [2.0, g["hi"][4] - g["lo"][4]]
    L = [levels_of(E[j], g["eps"][j]) for j in range(5)]
    return E, L, max(L), sum(L) + 2


def bounds5(g, c=1.0):
    """eps' of z (normalized) and kappa, the pads' upper bounds (eps plus half
    of eps', rounded up to a step of at most eps'/(l+1)) and the apex guard
    (one leaf xy side, normalized)."""
    E, L, Ls, _ = geometry5(g)
    ez = g["eps"][2] / E[2] / (c * (Ls + 1))
    ek = g["eps"][3] / (c * (Ls + 1))
    padz_max = g["eps"][2] / E[2] + ez / 2 + ez / (ELL + 1)
    padk_max = g["eps"][3] + ek / 2 + ek / (ELL + 1)
    return ez, ek, padz_max, padk_max, 2.0 ** -max(L[0], L[1])


def sector_of(yaw):
    return int(math.floor((yaw + math.pi / 4) / (math.pi / 2))) % 4


# ----------------------------------------------------------------------------
# Closed form
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_noise_free_matches_pass_through_the_pose(seed):
    g = synth.pose5dof(seed=seed, n=400, n_in=200, noise_deg=0.0)
    x, y, z, yaw, fs = map(float, g["truth"])
    E = [g["hi"][j] - g["lo"][j] for j in range(3)]
    t, f, _ = oracle.parametrize(P(g))
    s = sector_of(yaw)
    kap_true = math.tan(yaw - s * math.pi / 2)
    X, Y, Z = [(v - g["lo"][j]) / E[j] for j, v in enumerate((x, y, z))]
    for i in g["planted"]:
        # the paper's equations in user units
        w1, w2, w3, xi, eta = (float(col[i]) for col in g["cols"])
        r = math.hypot(w1 - x, w2 - y)
        assert abs((w3 - eta * fs * r) - z) <= 1e-9 * max(1.0, abs(z))
        v1, v2 = _rot(s, w1 - x, w2 - y)
        tt = xi * fs
        assert v1 + tt * v2 > 0
        assert abs((v2 - tt * v1) / (v1 + tt * v2) - kap_true) <= 1e-9
        # the oracle's normalized surface at the normalized truth
        W1, W2, xin, etan, W3 = t[i, 0], t[i, 1], t[i, 2], t[i, 3], f[i, 0]
        v1, v2 = _rot(s, W1 - X, W2 - Y)
        assert abs((W3 - etan * fs * math.hypot(v1, v2)) - Z) <= 1e-12
        tt = xin * fs
        assert abs((v2 - tt * v1) / (v1 + tt * v2) - kap_true) <= 1e-9


# ----------------------------------------------------------------------------
# 4-DoF is the case f = 1
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_f_equal_one_gives_the_4dof_problem(seed):
    g4 = synth.config("pose4dof_tiny", seed=seed)
    p4 = P(g4)
    lo = list(g4["lo"][:4]) + [1.0]
    hi = list(g4["hi"][:4]) + [1.0 + 2.0 ** -40]
    eps = list(g4["eps"][:4]) + [1.0]
    p5 = oracle.Problem("pose5dof", g4["cols"], lo, hi, eps)
    k4, k5 = oracle.constants(p4), oracle.constants(p5)
    assert k5["L"][4] == 0 and k5["B"] == k4["B"]
    # same root lattice (the f bound changes no power-of-two step here)
    a4 = oracle.parametrize(p4, root_canon=True)
    a5 = oracle.parametrize(p5, root_canon=True)
    assert np.array_equal(a4[0], a5[0]) and np.array_equal(a4[1], a5[1])
    c4 = oracle.all_leaf_counts(p4).astype(np.int64)
    c5 = oracle.all_leaf_counts(p5).astype(np.int64)
    # f in [1, 1 + 2^-40] holds f = 1: never fewer; equal unless a decision
    # sits within ~1e-12 of its threshold
    assert np.all(c5 >= c4)
    assert np.mean(c5 == c4) >= 0.999
    r4, r5 = oracle.solve(p4), oracle.solve(p5)
    assert (r4["count"], r4["leaf_index"]) == (r5["count"], r5["leaf_index"])
    assert np.array_equal(r4["inliers"], r5["inliers"])


# ----------------------------------------------------------------------------
# Predicate: sound and tight
# ----------------------------------------------------------------------------
def _cell5(L, m1, cc, g):
    """Normalized x, y, z box, kappa interval and user-unit f interval of a
    level-m1 cell."""
    h = [2.0 ** -min(m1, L[j]) for j in range(5)]
    box = [(cc[j] * h[j], (cc[j] + 1) * h[j]) for j in range(3)]
    kb = (2 * cc[3] * h[3] - 1, 2 * (cc[3] + 1) * h[3] - 1)
    Ef = g["hi"][4] - g["lo"][4]
    fb = (g["lo"][4] + Ef * (cc[4] * h[4]), g["lo"][4] + Ef * ((cc[4] + 1) * h[4]))
    return box, kb, fb, h


@pytest.mark.parametrize("name,seed", [("pose5dof_small", 17), ("pose5dof_small", 19), ("pose5dof_tiny", 7)])
def test_predicate_is_sound_and_tight(name, seed):
    g = synth.config(name, seed=seed)
    pr = P(g)
    E, L, Ls, B = geometry5(g)
    ez, ek, pzm, pkm, Rg = bounds5(g)
    epz = g["eps"][2] / E[2]
    ekap = g["eps"][3]
    t, f, _ = oracle.parametrize(pr, root_canon=True)
    rng = np.random.default_rng(seed)
    G, GF = 24, 9
    s = np.linspace(0.0, 1.0, G)
    sf = np.linspace(0.0, 1.0, GF)
    SX, SY, SF = (a.ravel() for a in np.meshgrid(s, s, sf, indexing="ij"))
    n_pass = n_k = n_sound = 0
    for trial in range(2500):
        i = int(rng.integers(0, t.shape[0]))
        m = int(rng.integers(0, Ls))
        m1 = m + 1
        sec = int(rng.integers(0, 4))
        W1, W2, xi, eta, W3 = t[i, 0], t[i, 1], t[i, 2], t[i, 3], f[i, 0]
        # a cell near the surface: a point of it, coordinates jittered
        X0, Y0, U0 = rng.uniform(0, 1, 3)
        F0 = g["lo"][4] + (g["hi"][4] - g["lo"][4]) * U0
        v1, v2 = _rot(sec, W1 - X0, W2 - Y0)
        D = v1 + xi * F0 * v2
        if D <= 0:
            continue
        kap = (v2 - xi * F0 * v1) / D
        Z = W3 - eta * F0 * math.hypot(v1, v2)
        n1 = [2 ** min(m1, L[j]) for j in range(5)]
        base = [X0, Y0, min(max(Z, 0.0), 1 - 1e-12), min(max((kap + 1) / 2, 0.0), 1 - 1e-12), U0]
        cc = [int(min(n1[j] - 1, max(0, math.floor(base[j] * n1[j]) + int(rng.integers(-2, 3)))))
              for j in range(5)]
        met = oracle.meets(pr, t[i], f[i], 0, m, sec, cc)
        box, (Klo, Khi), (Fl, Fh), h = _cell5(L, m1, cc, g)
        # z: exact range over the cell, from the ranges of r and of f
        ax0, ax1 = W1 - box[0][1], W1 - box[0][0]
        ay0, ay1 = W2 - box[1][1], W2 - box[1][0]
        rmin = math.hypot(max(0.0, ax0, -ax1), max(0.0, ay0, -ay1))
        rmax = math.hypot(max(abs(ax0), abs(ax1)), max(abs(ay0), abs(ay1)))
        prods = [eta * ff * rr for ff in (Fl, Fh) for rr in (rmin, rmax)]
        z0, z1 = W3 - max(prods), W3 - min(prods)
        zd = max(0.0, box[2][0] - z1, z0 - box[2][1])
        # kappa as an angle over a dense (x, y, f) grid of the cell
        X = box[0][0] + SX * h[0]
        Y = box[1][0] + SY * h[1]
        Fs = Fl + SF * (Fh - Fl)
        w1, w2 = _rot(sec, W1 - X, W2 - Y)
        T = xi * Fs
        Dg = w1 + T * w2
        psi = np.arctan2(w2 - T * w1, Dg)  # = atan(kappa) where D > 0
        if met:
            n_pass += 1
            assert zd <= pzm * (1 + 1e-9), (trial, zd, pzm)
            if rmin >= Rg:
                res = h[0] / (G - 1) * math.sqrt(2) / rmin + abs(xi) * (Fh - Fl) / (GF - 1) + 1e-12
                ok = (Dg > 0) & (psi >= math.atan(Klo - pkm) - res) & (psi <= math.atan(Khi + pkm) + res)
                assert ok.any(), (trial, i, m, sec, cc)
                n_k += 1
        else:
            # sound: within eps on z (exactly) and on kappa (at a sample)
            kok = (Dg > 0) & (psi >= math.atan(Klo - ekap)) & (psi <= math.atan(Khi + ekap))
            assert not (zd <= epz * (1 - 1e-9) and kok.any()), (trial, i, m, sec, cc)
            n_sound += 1
    assert n_pass > 150 and n_k > 60 and n_sound > 150


@pytest.mark.parametrize("name", ["pose5dof_small", "pose5dof_tiny"])
def test_root_lattice_moves_z_and_kappa_by_at_most_half_eps_prime(name):
    g = synth.config(name)
    pr = P(g)
    ez, ek, pzm, pkm, Rg = bounds5(g)
    t0, f0, _ = oracle.parametrize(pr)
    t1, f1, _ = oracle.parametrize(pr, root_canon=True)
    rng = np.random.default_rng(3)
    X, Y = rng.uniform(0, 1, (2, 4000))
    F = rng.uniform(g["lo"][4], g["hi"][4], 4000)
    worst_z = worst_k = 0.0
    kmax = 1.0 + g["eps"][3] + ek / 2
    for i in range(0, t0.shape[0], max(1, t0.shape[0] // 300)):
        for sec in range(4):
            va = _rot(sec, t0[i, 0] - X, t0[i, 1] - Y)
            vb = _rot(sec, t1[i, 0] - X, t1[i, 1] - Y)
            za = f0[i, 0] - t0[i, 3] * F * np.hypot(*va)
            zb = f1[i, 0] - t1[i, 3] * F * np.hypot(*vb)
            dz = float(np.max(np.abs(za - zb)))
            assert dz <= ez / 2 * (1 + 1e-6), (i, dz, ez / 2)
            worst_z = max(worst_z, dz / (ez / 2))
            Ta, Tb = t0[i, 2] * F, t1[i, 2] * F
            Da = va[0] + Ta * va[1]
            Db = vb[0] + Tb * vb[1]
            ka = (va[1] - Ta * va[0]) / np.where(Da > 0, Da, 1.0)
            kb = (vb[1] - Tb * vb[0]) / np.where(Db > 0, Db, 1.0)
            sel = (Da > 0) & (Db > 0) & (np.hypot(*va) >= Rg) & (np.abs(ka) <= kmax)
            if sel.any():
                dk = float(np.max(np.abs(ka - kb)[sel]))
                assert dk <= ek / 2 * 1.02, (i, sec, dk, ek / 2)
                worst_k = max(worst_k, dk / (ek / 2))
    assert worst_z > 0.05 and worst_k > 0.02


# ----------------------------------------------------------------------------
# Search
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [7, 8, 9])
def test_search_is_the_argmax_of_every_leaf(seed):
    g = synth.config("pose5dof_tiny", seed=seed)
    pr = P(g)
    E, L, Ls, B = geometry5(g)
    counts = oracle.all_leaf_counts(pr).astype(np.int64)
    assert counts.size == 1 << B
    r = oracle.solve(pr)
    best = int(np.argmax(counts))  # first maximum = lowest index
    assert (r["count"], r["leaf_index"]) == (int(counts[best]), best)
    for kw in (dict(no_prune=True), dict(no_group=True), dict(no_dive=True), dict(threads=4)):
        r2 = oracle.solve(P(g, **kw))
        assert (r2["count"], r2["leaf_index"]) == (r["count"], r["leaf_index"]), kw
        assert np.array_equal(r2["inliers"], r["inliers"])


def test_search_small_thread_pool_and_switches():
    g = synth.config("pose5dof_small")
    r = oracle.solve(P(g))
    for kw in (dict(threads=4), dict(no_dive=True)):
        r2 = oracle.solve(P(g, **kw))
        assert (r2["count"], r2["leaf_index"]) == (r["count"], r["leaf_index"]), kw
        assert np.array_equal(r2["inliers"], r["inliers"])


# ----------------------------------------------------------------------------
# (LOW) and (UP) at every leaf
# ----------------------------------------------------------------------------
def _leaf_boxes5(g, L):
    coords, sec = leaf_grid(L, True)
    E, *_ = geometry5(g)
    lo = np.array(list(g["lo"][:3]) + [-1.0, g["lo"][4]], float)
    h = np.array([E[j] * 2.0 ** -L[j] for j in range(5)])
    return lo + coords * h, lo + (coords + 1) * h, sec


def _pose5_parts(g, i, blo, bhi, sec):
    """From the match (w, xi, eta) itself, per leaf: the distance of its z
    range (metres) to the leaf's z interval, r_min, and the span of the
    angle atan(kappa) over the leaf's (x, y, f) box."""
    w1, w2, w3, xi, eta = (float(col[i]) for col in g["cols"])
    dx = np.maximum(0.0, np.maximum(blo[:, 0] - w1, w1 - bhi[:, 0]))
    dy = np.maximum(0.0, np.maximum(blo[:, 1] - w2, w2 - bhi[:, 1]))
    rmin = np.hypot(dx, dy)
    rmax = np.hypot(np.maximum(np.abs(w1 - blo[:, 0]), np.abs(w1 - bhi[:, 0])),
                    np.maximum(np.abs(w2 - blo[:, 1]), np.abs(w2 - bhi[:, 1])))
    prods = np.stack([eta * blo[:, 4] * rmin, eta * blo[:, 4] * rmax, eta * bhi[:, 4] * rmin,
                      eta * bhi[:, 4] * rmax])
    zmin, zmax = w3 - prods.max(0), w3 - prods.min(0)
    zdist = np.maximum(0.0, np.maximum(blo[:, 2] - zmax, zmin - bhi[:, 2]))
    a0, a1 = _angle_span(w1, w2, blo, bhi)
    o1, o2 = np.arctan(xi * blo[:, 4]), np.arctan(xi * bhi[:, 4])
    off = sec * (np.pi / 2)
    return zdist, rmin, a0 - off - np.maximum(o1, o2), a1 - off - np.minimum(o1, o2)


@pytest.mark.parametrize("seed", [7, 8])
def test_every_leaf_low_and_up(seed):
    g = synth.config("pose5dof_tiny", seed=seed)
    pr = P(g)
    E, L, Ls, B = geometry5(g)
    ez, ek, pzm, pkm, Rg = bounds5(g)
    blo, bhi, sec = _leaf_boxes5(g, L)
    n = len(g["cols"][0])
    total = np.zeros(blo.shape[0], np.int64)
    n_low = 0
    e3 = g["eps"][3]
    band = ek * Rg / (ELL + 1) * E[0]
    for i in range(n):
        ind = oracle.leaf_indicator(pr, i).astype(bool)
        total += ind
        zdist, rmin, p0, p1 = _pose5_parts(g, i, blo, bhi, sec)
        # LOW, per axis (z and kappa are tested separately)
        zlow = zdist <= g["eps"][2] * (1 - 1e-9)
        klow = _overlap_mod(p0, p1, np.arctan(blo[:, 3] - e3 * (1 - 1e-9)), np.arctan(bhi[:, 3] + e3 * (1 - 1e-9)))
        guard = rmin < Rg * E[0] - band
        low = zlow & (guard | ((rmin > Rg * E[0] + band) & klow))
        assert np.all(ind[low]), i
        n_low += int(low.sum())
        # UP: z within the pad bound plus the root quantization; kappa
        # likewise where the leaf is outside the apex guard
        assert np.all(zdist[ind] <= (pzm + ez / 2) * E[2] * (1 + 1e-9)), i
        kb = (pkm + ek / 2) * 1.02
        far = ind & (rmin >= Rg * E[0] * (1 + 1e-9))
        kup = _overlap_mod(p0, p1, np.arctan(blo[:, 3] - kb) - 1e-9, np.arctan(bhi[:, 3] + kb) + 1e-9)
        assert np.all(kup[far]), i
    assert np.array_equal(total, oracle.all_leaf_counts(pr).astype(np.int64))
    assert n_low > 0


def test_counts_shrink_down_the_tree():
    g = synth.config("pose5dof_tiny")
    pr = P(g)
    E, L, Ls, B = geometry5(g)
    n = len(g["cols"][0])
    prev = oracle.level_counts(pr, 0)
    assert np.all(prev == n) and prev.size == 4
    for m in range(Ls):
        cur = oracle.level_counts(pr, m + 1)
        a = sum(1 for j in range(5) if m < L[j])
        parent = np.repeat(prev, 1 << a)
        assert cur.size == parent.size
        assert np.all(cur <= parent), m
        prev = cur
    assert np.array_equal(prev, oracle.all_leaf_counts(pr))


# ----------------------------------------------------------------------------
# Returned point, levels
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["pose5dof_tiny", "pose5dof_small"])
def test_point_is_the_centre_of_the_returned_leaf(name):
    g = synth.config(name)
    E, L, Ls, B = geometry5(g)
    r = oracle.solve(P(g))
    sec, coords = decode_leaf(L, r["leaf_index"], True)
    assert list(r["leaf_coords"]) == coords and r["sector"] == sec
    for j in (0, 1, 2, 4):
        lo = g["lo"][j] + E[j] * coords[j] * 2.0 ** -L[j]
        hi = g["lo"][j] + E[j] * (coords[j] + 1) * 2.0 ** -L[j]
        assert abs(r["point"][j] - (lo + hi) / 2) <= 1e-12 * max(1.0, abs(hi))
    klo = -1.0 + 2.0 * coords[3] * 2.0 ** -L[3]
    khi = -1.0 + 2.0 * (coords[3] + 1) * 2.0 ** -L[3]
    assert 0.0 <= r["point"][3] < 2 * math.pi
    assert abs(math.tan(r["point"][3] - sec * math.pi / 2) - (klo + khi) / 2) <= 1e-12


@pytest.mark.parametrize("seed", [17, 19, 21])
def test_point_near_the_planted_truth(seed):
    """The chosen leaf holds at least as many surfaces as the truth's leaf,
    which holds every planted match within eps; the position and yaw lie
    within a few eps of the truth, and f within the ambiguity of a coarse
    eps (the pose and f trade off over the narrow bearing range)."""
    g = synth.config("pose5dof_small", seed=seed)
    pr = P(g)
    E, L, Ls, B = geometry5(g)
    r = oracle.solve(pr)
    tr = list(map(float, g["truth"]))
    for j in range(3):
        assert abs(r["point"][j] - tr[j]) <= 2 * g["eps"][j] + E[j] * 2.0 ** -L[j], (j, r["point"][j], tr[j])
    dyaw = abs(r["point"][3] - tr[3])
    assert min(dyaw, 2 * math.pi - dyaw) <= 4 * g["eps"][3]
    assert abs(r["point"][4] - tr[4]) <= 0.15 * tr[4]
    assert len(set(g["planted"].tolist()) & set(r["inliers"].tolist())) >= 0.95 * len(g["planted"])


def test_leaf_levels_of_the_benchmark_workload():
    g = synth.config("pose5dof_20k")
    E, L, Ls, B = geometry5(g)
    assert L == [8, 8, 5, 8, 7] and Ls == 8 and B == 38
    k = oracle.constants(P(g))
    assert k["L"] == L and k["Lstar"] == Ls and k["B"] == B


# a wide f range (f up to 2.6 times the truth, so that the f bound changes
# every step by at least a power of two) and a flat, coarse box in which the
# z bound, not the kappa bound, limits the W step
WIDE = dict(n=2000, n_in=200, noise_deg=0.2, half_z=10.0, rho=(2.0, 80.0), eps_m=4.0, eps_deg=2.0,
            eps_f_rel=0.05, f_range=(0.6, 2.6))
FLAT = dict(n=600, n_in=100, noise_deg=0.2, half_z=0.5, elev=1.0, rho=(2.0, 60.0), eps_m=50.0, eps_z=0.02,
            eps_deg=5.0, eps_f_rel=0.25, f_range=(0.6, 2.6))


def _config(name, seed):
    if name == "wide":
        return synth.pose5dof(seed=seed, **WIDE)
    if name == "flat":
        return synth.pose5dof(seed=seed, **FLAT)
    return synth.config(name, seed=seed)


@pytest.mark.parametrize("name,seed", [("pose5dof_small", s) for s in (17, 19, 21)] +
                         [("pose5dof_tiny", s) for s in (7, 8, 9)] + [("wide", s) for s in (31, 32, 33)] +
                         [("flat", s) for s in (41, 42, 43)])
def test_each_root_step_moves_z_and_kappa_by_at_most_its_share(name, seed):
    """Each of the l + 1 = 5 parameters that z (W1, W2, W3, xi, eta') and
    kappa (W1, W2, xi) depend on is rounded by at most half its step, which
    may move z or kappa by at most eps'/(2(l+1)) anywhere on the box: the
    worst case over the box of each parameter's own movement, from the
    derivatives dz/dW3 = 1, dz/deta' = f r, dz/dW = eta' f dr/dW (|dr/dW| <=
    1), dkappa/dxi = -(1 + kappa^2) f / (1 + t^2), dkappa/dW <= (1 +
    kappa^2)/r (r >= R_g), with f <= hi[4] and |kappa| <= 1 + eps_kappa + eps'/2.
    Each share is also used: the largest movement over the surfaces reaches a
    good part of it, so a needlessly fine step is caught too."""
    g = _config(name, seed)
    pr = P(g)
    ez, ek, pzm, pkm, Rg = bounds5(g)
    t0, f0, _ = oracle.parametrize(pr)
    t1, f1, _ = oracle.parametrize(pr, root_canon=True)
    fhi = g["hi"][4]
    kmax = 1.0 + g["eps"][3] + ek / 2
    Bk = 1.0 + kmax * kmax
    # farthest corner of the unit xy square from each surface's apex
    rmax = np.hypot(np.maximum(np.abs(t0[:, 0]), np.abs(t0[:, 0] - 1)),
                    np.maximum(np.abs(t0[:, 1]), np.abs(t0[:, 1] - 1)))
    eta = np.maximum(np.abs(t0[:, 3]), np.abs(t1[:, 3]))
    share_z, share_k = ez / (2 * (ELL + 1)), ek / (2 * (ELL + 1))
    moves = {
        "z/W3": np.abs(f1[:, 0] - f0[:, 0]) / share_z,
        "z/eta": np.abs(t1[:, 3] - t0[:, 3]) * fhi * (rmax + 2 ** -30) / share_z,
        "z/W1": np.abs(t1[:, 0] - t0[:, 0]) * eta * fhi / share_z,
        "z/W2": np.abs(t1[:, 1] - t0[:, 1]) * eta * fhi / share_z,
        "k/xi": np.abs(t1[:, 2] - t0[:, 2]) * Bk * fhi / share_k,
        "k/W1": np.abs(t1[:, 0] - t0[:, 0]) * Bk / Rg / share_k,
        "k/W2": np.abs(t1[:, 1] - t0[:, 1]) * Bk / Rg / share_k,
    }
    for what, v in moves.items():
        assert np.all(v <= 1.0 + 1e-6), (what, float(v.max()))
    # every step is as coarse as its own bound allows, up to the power of two
    # and the sampling of the rounding errors (W: the tighter of z and kappa)
    assert moves["z/W3"].max() > 0.35 and moves["z/eta"].max() > 0.25 and moves["k/xi"].max() > 0.35
    assert max(moves["z/W1"].max(), moves["k/W1"].max()) > 0.35
    if name == "flat":  # here the z bound is the one that limits the W step
        assert moves["z/W1"].max() > 0.35
