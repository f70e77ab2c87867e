"""Pins of the depth tracker oracle (section "Tracking": point-to-plane alignment
to the raycast surface over a resolution hierarchy), each against something other
than the oracle's own formulas:

* the depth hierarchy against a vectorised masked mean (brute force);
* the 6 x 6 solve against numpy, the rotation update against scipy's rotation
  vectors;
* the normal equations against finite differences of the energy: on a plane the
  point-to-plane distance does not depend on which reference pixel a point pairs
  with, so E(T) = sum d^2 is smooth, dE/dxi = 2 g and dg/dxi = A (Gauss-Newton,
  exact up to the rotation's curvature);
* recovery of a known rigid motion in a room corner (three orthogonal walls fix
  all six degrees of freedom), with exact analytic depth and reference maps.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

K = (140.0, 140.0, 79.5, 59.5)
W, H = 160, 120
CORNER = [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]]
FLOOR = [[0, 1, 0, 0]]
T_REF = synth.pose_look_at([1.5, 1.2, 1.8], [0.2, 0.2, 0.2], [0, 1, 0])


def moved(T, w, v):
    """(exp([w]x), v) T, built with scipy (independent of the oracle's update)."""
    Ri = Rotation.from_rotvec(w).as_matrix()
    out = np.eye(4)
    out[:3, :3] = Ri @ T[:3, :3]
    out[:3, 3] = Ri @ T[:3, 3] + np.asarray(v, np.float64)
    return out


def test_depth_level_brute_force():
    rng = np.random.default_rng(5)
    d = rng.uniform(0.5, 4.0, (61, 83)).astype(np.float32)
    d[rng.random(d.shape) < 0.3] = 0.0
    d[rng.random(d.shape) < 0.05] = np.nan
    d[rng.random(d.shape) < 0.05] = np.inf
    d[rng.random(d.shape) < 0.05] = -1.0
    clean = np.where(np.isfinite(d) & (d > 0), d.astype(np.float64), 0.0)
    for level in (0, 1, 2, 3):
        want = clean[:: 1 << level, :: 1 << level]
        got = oracle.depth_level(d, level)
        assert got.shape == want.shape == (-(-61 // (1 << level)), -(-83 // (1 << level)))
        assert np.array_equal(got, want)


def test_solve6_against_numpy():
    rng = np.random.default_rng(6)
    M = rng.standard_normal((6, 6))
    A = M @ M.T + 0.1 * np.eye(6)
    b = rng.standard_normal(6)
    up = np.concatenate([A[i, i:] for i in range(6)])
    np.testing.assert_allclose(oracle.solve6(up, b), np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.solve6(np.concatenate([(-A)[i, i:] for i in range(6)]), b)


def test_pose_step_against_rotation_vectors():
    rng = np.random.default_rng(7)
    for _ in range(5):
        xi = rng.standard_normal(6) * [0.3, 0.3, 0.3, 0.1, 0.1, 0.1]
        np.testing.assert_allclose(oracle.pose_step(xi, T_REF), moved(T_REF, xi[:3], xi[3:]), atol=1e-14)
    np.testing.assert_array_equal(oracle.pose_step(np.zeros(6), T_REF), T_REF)


def _floor_case():
    T_ref = synth.pose_look_at([0.3, 1.5, 0.2], [0.5, 0.0, 1.2], [0, 1, 0])
    _, V, N = synth.render_plane_maps(FLOOR, K, W, H, T_ref)
    T = moved(T_ref, [0.01, -0.02, 0.015], [0.01, 0.02, -0.01])
    depth = synth.render_plane_maps(FLOOR, K, W, H, T)[0].astype(np.float32)
    return depth, V, N, T_ref, T


@pytest.mark.parametrize("level", [0, 1])
def test_gradient_is_half_the_energy_derivative(level):
    depth, V, N, T_ref, T = _floor_case()
    s0 = oracle.icp_system(depth, K, level, V, N, T_ref, T, 1.0)
    assert s0[28] > 1000
    eps = 1e-7
    for i in range(6):
        e = np.zeros(6)
        e[i] = eps
        sp = oracle.icp_system(depth, K, level, V, N, T_ref, oracle.pose_step(e, T), 1.0)
        sm = oracle.icp_system(depth, K, level, V, N, T_ref, oracle.pose_step(-e, T), 1.0)
        assert sp[28] == sm[28] == s0[28]
        dE = (sp[27] - sm[27]) / (2 * eps)
        assert abs(dE - 2 * s0[21 + i]) <= 1e-5 * max(1.0, abs(dE)), (i, dE, 2 * s0[21 + i])


def test_hessian_is_the_gauss_newton_matrix():
    depth, V, N, T_ref, T = _floor_case()
    s0 = oracle.icp_system(depth, K, 0, V, N, T_ref, T, 1.0)
    A = np.zeros((6, 6))
    k = 0
    for i in range(6):
        for j in range(i, 6):
            A[i, j] = A[j, i] = s0[k]
            k += 1
    eps = 1e-6
    scale = np.abs(A).max()
    for j in range(6):
        e = np.zeros(6)
        e[j] = eps
        gp = oracle.icp_system(depth, K, 0, V, N, T_ref, oracle.pose_step(e, T), 1.0)[21:27]
        gm = oracle.icp_system(depth, K, 0, V, N, T_ref, oracle.pose_step(-e, T), 1.0)[21:27]
        col = (gp - gm) / (2 * eps)
        assert np.abs(col - A[:, j]).max() <= 2e-3 * scale, (j, col, A[:, j])


def test_recovers_a_known_motion():
    _, V, N = synth.render_plane_maps(CORNER, K, W, H, T_REF)
    T_true = moved(T_REF, [0.02, -0.03, 0.01], [0.03, -0.02, 0.025])
    depth = synth.render_plane_maps(CORNER, K, W, H, T_true)[0].astype(np.float32)
    T, info = oracle.track(depth, K, V, N, T_REF, T_REF, iters=(6, 6, 6), dist=(0.05, 0.1, 0.2))
    assert info["steps"] == 18 and info["pairs"] > 10000
    # not exact: points within a pixel of the corner's edges pair with the other
    # wall's reference pixel (projective pairing), which biases the optimum by
    # ~1e-5; the motion itself is 0.037 rad and 4.4 cm
    ang = np.linalg.norm(Rotation.from_matrix(T[:3, :3] @ T_true[:3, :3].T).as_rotvec())
    assert ang < 1e-4 and np.abs(T[:3, 3] - T_true[:3, 3]).max() < 1e-4, (ang, T[:3, 3] - T_true[:3, 3])
    assert info["rms"] < 2e-3
    # from the start the distances are ~100 times larger
    start = oracle.icp_system(depth, K, 0, V, N, T_REF, T_REF, 0.05)
    assert np.sqrt(start[27] / start[28]) > 50 * info["rms"]


def test_too_few_pairs_takes_no_step():
    _, V, N = synth.render_plane_maps(CORNER, K, W, H, T_REF)
    depth = synth.render_plane_maps(CORNER, K, W, H, moved(T_REF, [0, 0.01, 0], [0.01, 0, 0]))[0]
    T, info = oracle.track(depth.astype(np.float32), K, V, N, T_REF, T_REF, min_inliers=10 ** 9)
    assert info["steps"] == 0
    np.testing.assert_array_equal(T, T_REF)


def test_hierarchy_keeps_points_on_the_surface():
    """Level l back-projects pixel (u, v) as input pixel (2^l u, 2^l v), i.e. with
    fx / 2^l and cx / 2^l: at the pose the depth was taken from, every level's
    points lie on the floor to float32 depth rounding; a half-pixel slip of the
    principal point would put them millimetres off (the camera is rolled, so
    both image axes climb the floor).  And each point pairs with the reference
    pixel it came from."""
    T_ref = synth.pose_look_at([0.3, 1.5, 0.2], [0.5, 0.0, 1.2], [0.5, 1, 0])
    depth, V, N = synth.render_plane_maps(FLOOR, K, W, H, T_ref)
    for level in (0, 1, 2, 3):
        s = oracle.icp_system(depth.astype(np.float32), K, level, V, N, T_ref, T_ref, 1e-5)
        assert s[28] == (W >> level) * (H >> level)
        assert np.sqrt(s[27] / s[28]) < 1e-6, (level, np.sqrt(s[27] / s[28]))
