"""Pins of the oracle's verification and refinement after the vote (pose
families; Sec. 4.2: the vote's pose is taken by a more accurate method that
works on the nearly outlier-free inlier set; Sec. 5: the angular error of
the final inlier set is verified), against what geometry fixes, computed
here in world axes with the yaw angle and trigonometry (the oracle works in
the sector's frame with kappa, without trigonometry):

  * verification: the matches kept at the leaf centre are exactly those
    whose angle between the observed bearing and the direction to their
    point is at most tau0 (away from the threshold by more than 1e-9 rad);
  * refinement: on noise-free data it recovers the planted pose to rounding
    level and keeps every planted match; on noisy data the returned pose is
    a minimum of the sum of squared unit-direction differences over the
    returned set (no coordinate step lowers it) and lies nearer the truth
    than the leaf centre; zero rounds return the leaf centre.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_11810_amd import synth


def P(g, **kw):
    return oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"], **kw)


def world_dirs(g, pose, idx):
    """Observed bearing and direction to the point, in world axes, for pose
    (x, y, z, yaw[, f])."""
    x, y, z, yaw = pose[:4]
    f = pose[4] if g["family"] == "pose5dof" else 1.0
    w1, w2, w3, xi, eta = (np.asarray(c)[idx] for c in g["cols"])
    a, b = xi * f, eta * f
    h = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    lat = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
    up = np.array([0.0, 0.0, 1.0])
    obs = h[None, :] + a[:, None] * lat[None, :] + (b * np.sqrt(1 + a * a))[:, None] * up[None, :]
    pred = np.stack([w1 - x, w2 - y, w3 - z], axis=1)
    return obs, pred


def angles(g, pose, idx):
    o, d = world_dirs(g, pose, idx)
    cr = np.linalg.norm(np.cross(o, d), axis=1)
    return np.arctan2(cr, np.sum(o * d, axis=1))


def cost(g, pose, idx):
    o, d = world_dirs(g, pose, idx)
    r = d / np.linalg.norm(d, axis=1, keepdims=True) - o / np.linalg.norm(o, axis=1, keepdims=True)
    return float(np.sum(r * r))


def vote(g):
    pr = P(g)
    return pr, oracle.solve(pr)


@pytest.mark.parametrize("name,seed", [("pose4dof_small", 14), ("pose4dof_small", 15), ("pose5dof_small", 17),
                                       ("pose5dof_small", 19), ("pose5dof_tiny", 7)])
def test_first_verification_is_the_angle_at_the_leaf_centre(name, seed):
    g = synth.config(name, seed=seed)
    pr, r = vote(g)
    tau0 = math.radians(3.0)
    rf = oracle.refine(pr, r["leaf_index"], r["inliers"], tau0, math.radians(1.0), rounds=0)
    # zero rounds: the pose is the vote's leaf centre
    d = 5 if g["family"] == "pose5dof" else 4
    assert np.allclose(rf["pose"][:d], r["point"][:d], rtol=0, atol=1e-12)
    ang = angles(g, r["point"], r["inliers"])
    clear = np.abs(ang - tau0) > 1e-9
    kept = np.isin(r["inliers"], rf["verified"])
    assert np.array_equal(kept[clear], (ang <= tau0)[clear])
    assert 0 < kept.sum() < len(r["inliers"]) or name == "pose5dof_tiny"


@pytest.mark.parametrize("fam,seed", [("pose4dof", 1), ("pose4dof", 2), ("pose5dof", 3), ("pose5dof", 4)])
def test_noise_free_refinement_recovers_the_pose(fam, seed):
    if fam == "pose4dof":
        g = synth.pose4dof(seed=seed, n=3000, n_in=300, noise_deg=0.0, eps_m=4.0, eps_deg=2.0, rho_max=80.0)
    else:
        g = synth.pose5dof(seed=seed, n=3000, n_in=300, noise_deg=0.0, half_z=10.0, rho=(2.0, 80.0), eps_m=4.0,
                           eps_deg=2.0, eps_f_rel=0.05)
    pr, r = vote(g)
    rf = oracle.refine(pr, r["leaf_index"], r["inliers"], math.radians(6.0), math.radians(0.05), rounds=3, iters=10)
    tr = list(map(float, g["truth"]))
    for j in range(3):
        assert abs(rf["pose"][j] - tr[j]) <= 1e-7 * 200, (j, rf["pose"][j], tr[j])
    dyaw = abs(rf["pose"][3] - tr[3])
    assert min(dyaw, 2 * math.pi - dyaw) <= 1e-9
    if fam == "pose5dof":
        assert abs(rf["pose"][4] - tr[4]) <= 1e-9
    # every planted match the vote reported is kept
    assert set(g["planted"].tolist()) & set(r["inliers"].tolist()) <= set(rf["verified"].tolist())
    assert rf["rms"] <= 1e-9
    # the verified set is the angle test at the final pose
    ang = angles(g, rf["pose"], r["inliers"])
    kept = np.isin(r["inliers"], rf["verified"])
    clear = np.abs(ang - math.radians(0.05)) > 1e-9
    assert np.array_equal(kept[clear], (ang <= math.radians(0.05))[clear])


# (seeds whose vote lands in the planted pose's basin: with the coarse eps of
# these small problems some seeds' best leaf is another pose's)
@pytest.mark.parametrize("name,seed", [("pose4dof_small", 14), ("pose4dof_small", 16), ("pose5dof_small", 17),
                                       ("pose5dof_small", 23), ("pose5dof_small", 25)])
def test_refined_pose_is_a_minimum_and_nearer_the_truth(name, seed):
    g = synth.config(name, seed=seed)
    pr, r = vote(g)
    rf = oracle.refine(pr, r["leaf_index"], r["inliers"], math.radians(4.0), math.radians(1.5), rounds=3, iters=12)
    V = rf["verified"]
    assert len(V) >= 0.9 * len(g["planted"])
    q = np.array(rf["pose"], float)
    d = 5 if g["family"] == "pose5dof" else 4
    c0 = cost(g, q, V)
    # no coordinate step lowers the cost (a stationary point, to rounding)
    steps = [1e-3, 1e-3, 1e-3, 1e-5, 1e-5][:d]
    for j in range(d):
        for sgn in (-1, 1):
            qq = q.copy()
            qq[j] += sgn * steps[j]
            assert cost(g, qq, V) >= c0 * (1 - 1e-9), (j, sgn)
    # the leaf centre has the larger cost on the same set
    assert cost(g, np.array(r["point"], float), V) > c0
    assert abs(math.sqrt(c0 / len(V)) - rf["rms"]) <= 1e-9 * max(1.0, rf["rms"])
    tr = np.array(g["truth"], float)
    assert np.linalg.norm(q[:3] - tr[:3]) < np.linalg.norm(np.array(r["point"][:3]) - tr[:3])
    dy = lambda a: min(abs(a - tr[3]), 2 * math.pi - abs(a - tr[3]))  # noqa: E731
    assert dy(q[3]) < dy(r["point"][3])
    if d == 5:
        assert abs(q[4] - tr[4]) < abs(r["point"][4] - tr[4])


def test_refine_rejects_bad_arguments():
    g = synth.config("pose5dof_tiny")
    pr, r = vote(g)
    with pytest.raises(oracle.OracleError):
        oracle.refine(pr, r["leaf_index"], r["inliers"], 0.0, 0.1)
    with pytest.raises(oracle.OracleError):
        oracle.refine(pr, r["leaf_index"], np.array([len(g["cols"][0])]), 0.1, 0.1)
    g2 = synth.config("line2d_tiny")
    with pytest.raises(oracle.OracleError):
        oracle.refine(P(g2), 0, np.array([0]), 0.1, 0.1)
