"""Seeded synthetic workloads (planted-inlier data).

Only input generation lives here: no step of the voting method.  Both the
device path and the CPU oracle consume these arrays.  Every generator uses
``numpy.random.Generator(PCG64(seed))``.

Recipes (each stands in for a workload of the paper):
  * line2d / plane3d: uniform outliers in the unit square/cube and inliers on
    a fixed line/plane with vertical Gaussian noise (the line-fitting data of
    the hyperplane-fitting evaluation).
  * ray3d: rays through a common camera centre, perturbed in direction, plus
    uniformly random rays (ray intersection in 3-space).
  * pose4dof: 2D-3D matches seen from a gravity-aligned camera at a random
    position and yaw, plus random matches (stands in for the SfM query
    matches of the posing evaluation, which are not available).
  * pose5dof: the same with an unknown focal length: image coordinates are
    direction tangents divided by the camera's factor f* (stands in for the
    SfM query matches of the 5DoF evaluation: about 1e4-2e4 matches, camera
    within 50 m horizontally and 5 m vertically of the truth, f within
    [0.6, 1.3] of the truth).
  * sim2d: two planar point sets, part of one mapped into the other by a
    similarity with noise; every pair is a hypothetical correspondence
    (pointset alignment).
"""
from __future__ import annotations

import math

import numpy as np

FAMILY_IDS = {"line2d": 1, "plane3d": 2, "ray3d": 3, "pose4dof": 4, "sim2d": 5, "pose5dof": 6}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _problem(family, cols, lo, hi, eps, truth, planted, **extra):
    d = {"family": family, "cols": [np.ascontiguousarray(c, dtype=np.float64) for c in cols],
         "lo": list(map(float, lo)), "hi": list(map(float, hi)), "eps": list(map(float, eps)),
         "truth": truth, "planted": np.asarray(planted, dtype=np.int64)}
    d.update(extra)
    return d


def _shuffle(rng, cols, is_in):
    perm = rng.permutation(len(is_in))
    cols = [c[perm] for c in cols]
    planted = np.nonzero(is_in[perm])[0]
    return cols, planted


def line2d(seed=101, n=10_000, n_in=500, sigma=0.002, lo=(-1.0, -1.0), hi=(1.0, 2.0),
           eps=(0.005, 0.005)):
    """Points in [0,1]^2: inliers on y = a x + b (|a| <= 1) plus N(0, sigma^2)
    vertical noise, the rest uniform.  Dual axes (a, b)."""
    rng = _rng(seed)
    ang = rng.uniform(-math.pi / 4, math.pi / 4)
    a = math.tan(ang)
    ax, ay = rng.uniform(0.25, 0.75, size=2)
    b = ay - a * ax
    # x range where the line stays inside the unit square
    xs = [0.0, 1.0]
    if a != 0.0:
        xs = sorted([(0.0 - b) / a, (1.0 - b) / a])
    x0, x1 = max(0.0, xs[0]), min(1.0, xs[1])
    px, py = [], []
    while len(px) < n_in:
        x = rng.uniform(x0, x1)
        y = a * x + b + rng.normal(0.0, sigma)
        if 0.0 <= y <= 1.0:
            px.append(x)
            py.append(y)
    ox = rng.uniform(0.0, 1.0, size=n - n_in)
    oy = rng.uniform(0.0, 1.0, size=n - n_in)
    cols = [np.concatenate([px, ox]), np.concatenate([py, oy])]
    is_in = np.zeros(n, bool)
    is_in[:n_in] = True
    cols, planted = _shuffle(rng, cols, is_in)
    return _problem("line2d", cols, lo, hi, eps, truth=(a, b), planted=planted)


def plane3d(seed=102, n=1_000_000, n_in=10_000, sigma=0.001, lo=(-1.0, -1.0, -2.0),
            hi=(1.0, 1.0, 3.0), eps=(0.003, 0.003, 0.003)):
    """Points in [0,1]^3: inliers on z = a0 + a1 x + a2 y (|a_i| <= 1) with
    N(0, sigma^2) vertical noise, the rest uniform.  Dual axes (a1, a2, a0)."""
    rng = _rng(seed)
    a1, a2 = rng.uniform(-1.0, 1.0, size=2)
    anc = rng.uniform(0.25, 0.75, size=3)
    a0 = anc[2] - a1 * anc[0] - a2 * anc[1]
    px = np.empty(0)
    py = np.empty(0)
    pz = np.empty(0)
    while px.size < n_in:
        m = 2 * (n_in - px.size) + 16
        x = rng.uniform(0.0, 1.0, size=m)
        y = rng.uniform(0.0, 1.0, size=m)
        z = a0 + a1 * x + a2 * y + rng.normal(0.0, sigma, size=m)
        ok = (z >= 0.0) & (z <= 1.0)
        px = np.concatenate([px, x[ok]])
        py = np.concatenate([py, y[ok]])
        pz = np.concatenate([pz, z[ok]])
    px, py, pz = px[:n_in], py[:n_in], pz[:n_in]
    o = rng.uniform(0.0, 1.0, size=(3, n - n_in))
    cols = [np.concatenate([px, o[0]]), np.concatenate([py, o[1]]), np.concatenate([pz, o[2]])]
    is_in = np.zeros(n, bool)
    is_in[:n_in] = True
    cols, planted = _shuffle(rng, cols, is_in)
    return _problem("plane3d", cols, lo, hi, eps, truth=(a1, a2, a0), planted=planted)


def _perp_basis(u):
    """Two unit vectors orthogonal to each row of u (n x 3)."""
    helper = np.where(np.abs(u[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    e1 = np.cross(u, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(u, e1)
    return e1, e2


def _perturb(rng, u, deg):
    e1, e2 = _perp_basis(u)
    g = rng.normal(0.0, 1.0, size=(u.shape[0], 2))
    s = math.tan(math.radians(deg))
    v = u + s * (g[:, :1] * e1 + g[:, 1:] * e2)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def ray3d(seed=103, n=100_000, n_in=1000, noise_deg=0.5, size=100.0, eps=0.25):
    """Rays w + s u in a cube: inliers point at a common centre c* (direction
    perturbed by a tangent-plane Gaussian of scale tan(noise_deg)), the rest
    have uniform origins and uniform directions.  Axes (x, y, z)."""
    rng = _rng(seed)
    c = rng.uniform(0.0, size, size=3)
    w_in = np.empty((0, 3))
    while w_in.shape[0] < n_in:
        w = rng.uniform(0.0, size, size=(2 * n_in, 3))
        ok = np.linalg.norm(c[None, :] - w, axis=1) >= 1.0
        w_in = np.concatenate([w_in, w[ok]])
    w_in = w_in[:n_in]
    u_in = c[None, :] - w_in
    u_in /= np.linalg.norm(u_in, axis=1, keepdims=True)
    u_in = _perturb(rng, u_in, noise_deg)
    w_out = rng.uniform(0.0, size, size=(n - n_in, 3))
    u_out = rng.normal(0.0, 1.0, size=(n - n_in, 3))
    u_out /= np.linalg.norm(u_out, axis=1, keepdims=True)
    W = np.concatenate([w_in, w_out])
    U = np.concatenate([u_in, u_out])
    cols = [W[:, 0], W[:, 1], W[:, 2], U[:, 0], U[:, 1], U[:, 2]]
    is_in = np.zeros(n, bool)
    is_in[:n_in] = True
    cols, planted = _shuffle(rng, cols, is_in)
    return _problem("ray3d", cols, (0.0, 0.0, 0.0), (size, size, size), (eps, eps, eps),
                    truth=tuple(c), planted=planted)


def bearing_to_xi_eta(d, yaw):
    """Gravity-aligned camera with heading (cos yaw, sin yaw): xi = lateral /
    forward (lateral = heading turned +90 deg about up), eta = vertical over
    horizontal distance (elevation tangent)."""
    h = np.array([math.cos(yaw), math.sin(yaw)])
    l = np.array([-math.sin(yaw), math.cos(yaw)])
    F = d[:, 0] * h[0] + d[:, 1] * h[1]
    L = d[:, 0] * l[0] + d[:, 1] * l[1]
    r = np.hypot(d[:, 0], d[:, 1])
    return L / F, d[:, 2] / r, F


def pose4dof(seed=104, n=1_000_000, n_in=5000, noise_deg=0.5, size=200.0, eps_m=0.5,
             eps_deg=0.5, rho_max=None, height=None):
    """2D-3D matches (w, xi, eta) for a camera at c* with yaw theta*: inliers
    are points seen at lateral tangent xi0 and elevation tangent eta0 in
    [-1, 1], horizontal range U(1, rho_max), bearing perturbed by noise_deg;
    outliers have uniform w and uniform (xi, eta) in [-1, 1]^2.
    Axes (x, y, z, yaw)."""
    rng = _rng(seed)
    rho_max = size if rho_max is None else rho_max
    height = size if height is None else height
    top = np.array([size, size, height])
    c = rng.uniform(0.0, top, size=3)
    yaw = rng.uniform(0.0, 2 * math.pi)
    ws, xis, etas = [], [], []
    got = 0
    tried = 0
    while got < n_in:
        if tried > 40 * n_in + 4000 and got < 0.01 * tried:
            # the camera sees (almost) none of the box from this pose, e.g. on
            # a wall facing out: draw another pose
            c = rng.uniform(0.0, top, size=3)
            yaw = rng.uniform(0.0, 2 * math.pi)
            ws, xis, etas = [], [], []
            got = tried = 0
        m = 4 * (n_in - got) + 16
        tried += m
        xi0 = rng.uniform(-1.0, 1.0, size=m)
        eta0 = rng.uniform(-1.0, 1.0, size=m)
        rho = rng.uniform(1.0, rho_max, size=m)
        hx = math.cos(yaw) - xi0 * math.sin(yaw)
        hy = math.sin(yaw) + xi0 * math.cos(yaw)
        nrm = np.sqrt(1.0 + xi0 * xi0)
        d = np.stack([rho * hx / nrm, rho * hy / nrm, rho * eta0], axis=1)
        w = c[None, :] + d
        ok = np.all((w >= 0.0) & (w <= top[None, :]), axis=1)
        w, d = w[ok], d[ok]
        if w.shape[0] == 0:
            continue
        dn = _perturb(rng, d / np.linalg.norm(d, axis=1, keepdims=True), noise_deg)
        xi, eta, F = bearing_to_xi_eta(dn, yaw)
        keep = F > 0
        ws.append(w[keep])
        xis.append(xi[keep])
        etas.append(eta[keep])
        got += int(keep.sum())
    w_in = np.concatenate(ws)[:n_in]
    xi_in = np.concatenate(xis)[:n_in]
    eta_in = np.concatenate(etas)[:n_in]
    w_out = rng.uniform(0.0, top, size=(n - n_in, 3))
    xi_out = rng.uniform(-1.0, 1.0, size=n - n_in)
    eta_out = rng.uniform(-1.0, 1.0, size=n - n_in)
    W = np.concatenate([w_in, w_out])
    cols = [W[:, 0], W[:, 1], W[:, 2], np.concatenate([xi_in, xi_out]), np.concatenate([eta_in, eta_out])]
    is_in = np.zeros(n, bool)
    is_in[:n_in] = True
    cols, planted = _shuffle(rng, cols, is_in)
    eps_k = math.radians(eps_deg)
    return _problem("pose4dof", cols, (0.0, 0.0, 0.0, 0.0), (size, size, height, 2 * math.pi),
                    (eps_m, eps_m, eps_m, eps_k), truth=(c[0], c[1], c[2], yaw), planted=planted)


def pose5dof(seed=106, n=20_000, n_in=300, noise_deg=0.5, half_xy=50.0, half_z=5.0, rho=(2.0, 100.0),
             elev=0.5, eps_m=0.5, eps_deg=0.5, eps_f_rel=0.01, f_range=(0.6, 1.3), eps_z=None):
    """2D-3D matches (w, xi, eta) for a gravity-aligned camera at c* with yaw
    theta* and an unknown focal length: the camera's direction tangents are
    f* times its image coordinates (f* = reference focal / true focal, drawn
    in [0.7, 1.4]).  Inliers: points at horizontal range U(rho), lateral
    tangent U(-1, 1), elevation tangent U(-elev, elev), bearing perturbed by
    noise_deg, observed at (xi, eta) = tangents / f*.  Outliers: points
    uniform over the region the inliers span, image coordinates uniform over
    the same image.  Axes (x, y, z, yaw, f): a box of 2 half_xy by 2 half_xy
    by 2 half_z around the camera, the truth uniform in its middle half, and
    f in [f_range] times f*."""
    rng = _rng(seed)
    c = np.array([rng.uniform(-100.0, 100.0), rng.uniform(-100.0, 100.0), rng.uniform(0.0, 20.0)])
    yaw = rng.uniform(0.0, 2 * math.pi)
    fstar = rng.uniform(0.7, 1.4)
    # box corner on a 2^-10 grid, so that hi - lo is exactly the box side
    lo_xyz = np.round((c - np.array([half_xy, half_xy, half_z]) * rng.uniform(0.5, 1.5, size=3)) * 1024.0) / 1024.0
    xi0 = rng.uniform(-1.0, 1.0, size=n_in)
    eta0 = rng.uniform(-elev, elev, size=n_in)
    r = rng.uniform(rho[0], rho[1], size=n_in)
    hx = math.cos(yaw) - xi0 * math.sin(yaw)
    hy = math.sin(yaw) + xi0 * math.cos(yaw)
    nrm = np.sqrt(1.0 + xi0 * xi0)
    d = np.stack([r * hx / nrm, r * hy / nrm, r * eta0], axis=1)
    w_in = c[None, :] + d
    dn = _perturb(rng, d / np.linalg.norm(d, axis=1, keepdims=True), noise_deg)
    xi_in, eta_in, F = bearing_to_xi_eta(dn, yaw)
    assert np.all(F > 0)
    m = n - n_in
    ang = rng.uniform(0.0, 2 * math.pi, size=m)
    ro = rho[1] * np.sqrt(rng.uniform((rho[0] / rho[1]) ** 2, 1.0, size=m))
    w_out = np.stack([c[0] + ro * np.cos(ang), c[1] + ro * np.sin(ang),
                      c[2] + ro * rng.uniform(-elev, elev, size=m)], axis=1)
    xi_out = rng.uniform(-1.0, 1.0, size=m)
    eta_out = rng.uniform(-elev, elev, size=m)
    W = np.concatenate([w_in, w_out])
    cols = [W[:, 0], W[:, 1], W[:, 2], np.concatenate([xi_in, xi_out]) / fstar,
            np.concatenate([eta_in, eta_out]) / fstar]
    is_in = np.zeros(n, bool)
    is_in[:n_in] = True
    cols, planted = _shuffle(rng, cols, is_in)
    hi_xyz = lo_xyz + np.array([2 * half_xy, 2 * half_xy, 2 * half_z])
    flo, fhi = f_range[0] * fstar, f_range[1] * fstar
    return _problem("pose5dof", cols, (lo_xyz[0], lo_xyz[1], lo_xyz[2], 0.0, flo),
                    (hi_xyz[0], hi_xyz[1], hi_xyz[2], 2 * math.pi, fhi),
                    (eps_m, eps_m, eps_m if eps_z is None else eps_z, math.radians(eps_deg), eps_f_rel * fstar),
                    truth=(c[0], c[1], c[2], yaw, fstar), planted=planted)


def sim2d(seed=105, n_a=10_000, k=9, n_in=1000, sigma=0.002, eps=0.01, lo=(0.25, -1.25, -2.0, -2.0),
          hi=(1.25, 1.25, 2.0, 2.0)):
    """Point sets A, B in [0,1]^2 and k candidate correspondences per point
    of A, as a descriptor matcher would propose them.  n_in points of A (in
    [0.25, 0.75]^2) map into B by q = [[a, b], [-b, a]] p + (c, d), a =
    s cos t, b = s sin t, scale s in [0.6, 1.2], rotation t in [-60, 60]
    deg, plus isotropic Gaussian noise sigma, and their true image is one of
    their candidates; every other candidate is a uniform point.
    Observations: columns (px, py, qx, qy), n_a * k of them.  Axes
    (a, b, c, d); the box keeps a >= 0.25, away from the degenerate
    similarities of scale near 0 that map all of A to one point."""
    rng = _rng(seed)
    s = rng.uniform(0.6, 1.2)
    t = rng.uniform(-math.pi / 3, math.pi / 3)
    a, b = s * math.cos(t), s * math.sin(t)
    M = np.array([[a, b], [-b, a]])
    A = rng.uniform(0.0, 1.0, size=(n_a, 2))
    A[:n_in] = rng.uniform(0.25, 0.75, size=(n_in, 2))
    img = A[:n_in] @ M.T
    lo_t = -img.min(axis=0)
    hi_t = 1.0 - img.max(axis=0)
    tr = rng.uniform(lo_t, np.maximum(lo_t, hi_t))
    Q = rng.uniform(0.0, 1.0, size=(n_a, k, 2))
    slot = rng.integers(0, k, size=n_in)
    Q[np.arange(n_in), slot] = img + tr + rng.normal(0.0, sigma, size=(n_in, 2))
    P = np.repeat(A[:, None, :], k, axis=1)
    is_in = np.zeros((n_a, k), bool)
    is_in[np.arange(n_in), slot] = True
    cols = [P[..., 0].ravel(), P[..., 1].ravel(), Q[..., 0].ravel(), Q[..., 1].ravel()]
    cols, planted = _shuffle(rng, cols, is_in.ravel())
    return _problem("sim2d", cols, lo, hi, (eps, eps, eps, eps), truth=(a, b, float(tr[0]), float(tr[1])),
                    planted=planted)


# --------------------------------------------------------------------------
# Named workloads.  Full sizes are the paper-scale planted-inlier configs; the
# "tiny" ones have few surfaces and a coarse eps so every leaf can be checked.
# --------------------------------------------------------------------------
def config(name: str, **kw):
    if name == "line2d_10k":
        return line2d(**kw)
    if name == "plane3d_1m":
        return plane3d(**kw)
    if name == "ray3d_100k":
        return ray3d(**kw)
    if name == "pose4dof_1m":
        return pose4dof(**kw)
    if name == "pose5dof_20k":
        return pose5dof(**kw)
    if name == "pose5dof_tiny":
        return pose5dof(seed=kw.get("seed", 7), n=kw.get("n", 48), n_in=kw.get("n_in", 12), noise_deg=0.2,
                        half_z=25.0, rho=(2.0, 60.0), eps_m=25.0, eps_deg=11.5, eps_f_rel=0.25)
    if name == "pose5dof_small":
        return pose5dof(seed=kw.get("seed", 17), n=kw.get("n", 3000), n_in=kw.get("n_in", 300), noise_deg=0.2,
                        half_z=10.0, rho=(2.0, 80.0), eps_m=4.0, eps_deg=2.0, eps_f_rel=0.05)
    if name == "sim2d_90k":
        return sim2d(**kw)
    if name == "sim2d_tiny":
        return sim2d(seed=kw.get("seed", 6), n_a=12, k=4, n_in=6, sigma=0.01, eps=0.3)
    if name == "sim2d_small":
        return sim2d(seed=kw.get("seed", 16), n_a=500, k=6, n_in=80, sigma=0.003, eps=0.03)
    if name == "line2d_tiny":
        return line2d(seed=kw.get("seed", 1), n=kw.get("n", 48), n_in=kw.get("n_in", 12), sigma=0.01,
                      eps=(0.1, 0.1))
    if name == "plane3d_tiny":
        return plane3d(seed=kw.get("seed", 2), n=kw.get("n", 48), n_in=kw.get("n_in", 12), sigma=0.01,
                       eps=(0.2, 0.2, 0.2))
    if name == "ray3d_tiny":
        return ray3d(seed=kw.get("seed", 3), n=kw.get("n", 48), n_in=kw.get("n_in", 12), noise_deg=0.5,
                     eps=12.0)
    if name == "pose4dof_tiny":
        return pose4dof(seed=kw.get("seed", 4), n=kw.get("n", 48), n_in=kw.get("n_in", 12), noise_deg=0.2,
                        eps_m=25.0, eps_deg=11.5, rho_max=60.0)
    if name == "pose4dof_tiny_flat":  # z extent smaller than the xy extent
        return pose4dof(seed=kw.get("seed", 5), n=kw.get("n", 48), n_in=kw.get("n_in", 12), noise_deg=0.2,
                        eps_m=25.0, eps_deg=11.5, rho_max=60.0, height=100.0)
    if name == "pose4dof_small_flat":
        return pose4dof(seed=kw.get("seed", 18), n=kw.get("n", 3000), n_in=kw.get("n_in", 300), noise_deg=0.2,
                        eps_m=4.0, eps_deg=2.0, rho_max=80.0, height=60.0)
    if name == "line2d_small":
        return line2d(seed=kw.get("seed", 11), n=kw.get("n", 2000), n_in=kw.get("n_in", 200), sigma=0.003,
                      eps=(0.01, 0.01))
    if name == "plane3d_small":
        return plane3d(seed=kw.get("seed", 12), n=kw.get("n", 2000), n_in=kw.get("n_in", 300), sigma=0.004,
                       eps=(0.04, 0.04, 0.04))
    if name == "ray3d_small":
        return ray3d(seed=kw.get("seed", 13), n=kw.get("n", 3000), n_in=kw.get("n_in", 300), noise_deg=0.2,
                     eps=1.0)
    if name == "pose4dof_small":
        return pose4dof(seed=kw.get("seed", 14), n=kw.get("n", 3000), n_in=kw.get("n_in", 300), noise_deg=0.2,
                        eps_m=4.0, eps_deg=2.0, rho_max=80.0)
    raise KeyError(name)


def batch_pose4dof(n_problems=256, base_seed=10_000, nmin=1_000, nmax=200_000, rmin=0.002, rmax=0.1,
                   meta_seed=199):
    """Many independent POSE4DOF problems of uneven size: N log-uniform in
    [nmin, nmax], inlier ratio log-uniform in [rmin, rmax]."""
    out = []
    for i in range(n_problems):
        r = _rng(base_seed + i)
        N = int(round(math.exp(r.uniform(math.log(nmin), math.log(nmax)))))
        ratio = math.exp(r.uniform(math.log(rmin), math.log(rmax)))
        n_in = max(3, int(round(N * ratio)))
        out.append(pose4dof(seed=base_seed + i, n=N, n_in=n_in))
    return out


def poisson_arrivals(n, rate, seed=199):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    r = _rng(seed)
    return np.cumsum(r.exponential(1.0 / rate, size=n))
