"""Pins of the oracle's voxel update, section "Integration"
(computeUpdatedVoxelDepthInfo), on single voxels seen by a camera at the origin.

Expectations are closed forms in exact rational arithmetic of the binary32 inputs:
a voxel v at world v*s seen from the identity pose has camera depth v_z*s, so
eta = d - v_z*s and f = min(1, eta/mu)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

S, MU = 0.01, 0.04
K = (100.0, 100.0, 50.0, 50.0)      # 101 x 101 image, principal point at pixel (50, 50)
W = H = 101


def f32(x):
    return Fr(float(np.float32(x)))


def expected_f(d, vz):
    eta = f32(d) - vz * f32(S)
    return min(Fr(1), eta / f32(MU))


def run(orc, depths, vox, max_w=100, Wimg=W, Himg=H, img=None):
    sc = orc.Scene(S, MU, max_w, 16, 4)
    vox = np.array(vox, np.int32).reshape(-1, 3)
    F = np.ones(len(vox))
    Wt = np.zeros(len(vox), np.int32)
    n = []
    for d in depths:
        im = np.full((Himg, Wimg), d, np.float32) if img is None else img(d)
        n.append(sc.update_voxels(im, K, np.eye(4), vox, np.ones(len(vox), np.uint8), F, Wt))
    return F, Wt, n


def test_single_update_values(orc):
    # voxel on the optical axis at 1.0 m (v = (0, 0, 100)); band mu = 4 cm
    for d in (1.01, 1.02, 0.995, 0.97, 1.5, 1.0):
        F, Wt, n = run(orc, [d], [(0, 0, 100)])
        assert n == [1] and Wt[0] == 1
        assert abs(F[0] - float(expected_f(d, 100))) < 1e-12


def test_behind_band_is_skipped(orc):
    # eta < -mu: no new information, nothing written
    F, Wt, n = run(orc, [0.95], [(0, 0, 100)])
    assert n == [0] and Wt[0] == 0 and F[0] == 1.0
    # the boundary eta = -mu exactly (d = 0.96 is not exact in binary32, so use the
    # voxel one band-width behind an exactly representable depth)
    F, Wt, n = run(orc, [1.0], [(0, 0, 104)])
    eta = f32(1.0) - 104 * f32(S)
    assert (n == [1]) == (eta >= -f32(MU))


def test_running_average_is_mean_below_cap(orc):
    depths = [1.01, 0.99, 1.03, 1.0, 1.025, 0.975]
    F, Wt, n = run(orc, depths, [(0, 0, 100)], max_w=1000)
    mean = sum(expected_f(d, 100) for d in depths) / len(depths)
    assert Wt[0] == len(depths)
    assert abs(F[0] - float(mean)) < 1e-12


def test_running_average_at_weight_cap(orc):
    # max_w = 1: after the first update every new value is averaged 1:1 with the
    # old one (W + 1 = 2 before the cap), so F_n = f_n/2 + f_{n-1}/4 + ... + f_1/2^(n-1)
    depths = [1.01, 0.99, 1.03, 1.0, 1.025]
    F, Wt, n = run(orc, depths, [(0, 0, 100)], max_w=1)
    fs = [expected_f(d, 100) for d in depths]
    m = len(fs)
    closed = fs[0] / 2 ** (m - 1) + sum(fs[k] / 2 ** (m - k) for k in range(1, m))
    assert Wt[0] == 1
    assert abs(F[0] - float(closed)) < 1e-12
    # max_w = 3 over 6 updates: W saturates at 3
    F, Wt, n = run(orc, depths + [1.0], [(0, 0, 100)], max_w=3)
    assert Wt[0] == 3


def test_invalid_depth_and_behind_camera(orc):
    for bad in (0.0, -1.0, np.nan, np.inf):
        F, Wt, n = run(orc, [bad], [(0, 0, 100)])
        assert n == [0] and Wt[0] == 0
    # voxel behind the camera (z <= 0) is skipped
    F, Wt, n = run(orc, [1.0], [(0, 0, -5), (0, 0, 0)])
    assert n == [0]


def test_image_border_and_nearest_pixel(orc):
    # voxels at 2 m depth (v_z = 200): image x = 50 + 100 * (v_x * s) / 2 = 50 + v_x / 2.
    # Border rule: skipped when x < 1 or x > W - 2 = 99; nearest pixel (int)(x + 0.5).
    cases = {(-99, 0, 200): None,   # x = 0.5  -> skipped
             (-98, 0, 200): 1,      # x = 1.0  -> pixel 1
             (-97, 0, 200): 2,      # x = 1.5  -> pixel 2
             (97, 0, 200): 99,      # x = 98.5 -> pixel 99
             (99, 0, 200): None}    # x = 99.5 -> skipped
    im = np.full((H, W), 2.0, np.float32)
    im[:, 1], im[:, 2], im[:, 99] = 2.01, 2.02, 2.03
    for v, px in cases.items():
        sc = orc.Scene(S, MU, 100, 16, 4)
        F = np.ones(1)
        Wt = np.zeros(1, np.int32)
        n = sc.update_voxels(im, K, np.eye(4), np.array([v], np.int32), np.ones(1, np.uint8), F, Wt)
        if px is None:
            assert n == 0, v
        else:
            assert n == 1, v
            eta = f32(im[0, px]) - v[2] * f32(S)
            assert abs(F[0] - float(min(Fr(1), eta / f32(MU)))) < 1e-12, (v, px)


# -- decision margins under a rotated pose -----------------------------------
# A GPU takes the update's integer decisions (nearest pixel, border, band) in
# binary32; within its error bound of a threshold both outcomes are correct.
# The oracle evaluates the definition in binary64 and keeps every outcome within
# the bound.  The voxels below are placed exactly on a threshold (the camera
# point chosen first, the pose solved for it), so the oracle must return both
# outcomes, with the values worked out here; a voxel well away from any
# threshold has one.

def rotated_pose_through(v, s, p_cam):
    """T_wc of a rotated camera that sees world point v*s at camera point p_cam"""
    from scipy.spatial.transform import Rotation
    R_cw = Rotation.from_rotvec([0.3, -0.2, 0.45]).as_matrix()
    s = float(np.float32(s))     # the voxel size as the scene holds it (binary32)
    t_cw = np.asarray(p_cam, np.float64) - R_cw @ (np.asarray(v, np.float64) * s)
    T = np.eye(4)
    T[:3, :3] = R_cw.T
    T[:3, 3] = -R_cw.T @ t_cw
    return T


S2, MU2 = 0.01, 0.0625           # mu = 1/16 exactly
K2 = (100.0, 100.0, 40.0, 30.0)  # 80 x 60 image
VOX = (37, -12, 91)


def outcomes(orc, img, p_cam):
    sc = orc.Scene(S2, MU2, 100, 16, 4)
    T = rotated_pose_through(VOX, S2, p_cam)
    got, unresolved = sc.voxel_outcomes(img, K2, T, np.array(VOX, np.int32))
    assert not unresolved
    return got, T


def depth_image(d=1.015625):
    return np.full((60, 80), d, np.float32)


def test_nearest_pixel_tie_keeps_both_pixels(orc):
    # x = 100 * 0.125 / 1 + 40 = 52.5: x + 1/2 = 53 lies on the rounding boundary
    # between pixels 52 and 53 (y = 36.25 is not on one)
    img = depth_image()
    img[36, 52] = 1.015625       # f = (1 + 1/64 - 1) / (1/16) = 1/4
    img[36, 53] = 1.0078125      # f = 1/8
    img[36, 54] = 1.0234375      # the wrong neighbour: f = 3/8
    img[36, 51] = 1.0234375
    got, _ = outcomes(orc, img, (0.125, 0.0625, 1.0))
    assert len(got) == 2 and all(u for u, _ in got)
    assert sorted(round(f, 12) for _, f in got) == [0.125, 0.25]
    # a point a tenth of a pixel away from the boundary: one outcome, pixel 53
    got, _ = outcomes(orc, img, (0.126, 0.0625, 1.0))
    assert len(got) == 1 and abs(got[0][1] - 0.125) < 1e-12
    # the tie on y: y = 100 * 0.065 / 1 + 30 = 36.5
    img2 = depth_image()
    img2[37, 53] = 1.0078125
    got, _ = outcomes(orc, img2, (0.126, 0.065, 1.0))
    assert sorted(round(f, 12) for _, f in got) == [0.125, 0.25]


def test_border_tie_keeps_skip_and_update(orc):
    # x = 100 * (-0.39) / 1 + 40 = 1, the border: inside (pixel 1) or skipped
    img = depth_image()
    img[36, 1] = 1.0078125
    got, _ = outcomes(orc, img, (-0.39, 0.0625, 1.0))
    assert sorted((u, round(f, 12)) for u, f in got) == [(False, 0.0), (True, 0.125)]
    # the far border x = W - 2 = 78: 100 * 0.38 + 40
    img[36, 78] = 1.0078125
    got, _ = outcomes(orc, img, (0.38, 0.0625, 1.0))
    assert sorted((u, round(f, 12)) for u, f in got) == [(False, 0.0), (True, 0.125)]


def test_band_tie_keeps_skip_and_update(orc):
    # eta = d - z = 0.9375 - 1 = -1/16 = -mu: updated with f = -1, or skipped
    img = depth_image(0.9375)
    got, _ = outcomes(orc, img, (0.126, 0.0625, 1.0))
    assert sorted((u, round(f, 12)) for u, f in got) == [(False, 0.0), (True, -1.0)]
    # a little further in front: one outcome
    got, _ = outcomes(orc, depth_image(0.9453125), (0.126, 0.0625, 1.0))
    assert got == [(True, -0.875)] or (len(got) == 1 and abs(got[0][1] + 0.875) < 1e-12)


def test_scene_keeps_the_other_state_until_the_next_frames(orc):
    """Integrated in a scene, the tie voxel carries two states (W = 1, F = 1/4 or
    1/8); a second frame without a tie moves both by the same update."""
    img = depth_image()
    img[36, 53] = 1.0078125
    p = (0.125, 0.0625, 1.0)
    T = rotated_pose_through(VOX, S2, p)
    sc = orc.Scene(S2, MU2, 100, 1 << 10, 1 << 8)
    sc.integrate(img, K2, T)
    c, F, W = sc.export()
    blk = tuple(np.floor_divide(VOX, 8))
    li = int(np.mod(VOX[0], 8) + 8 * np.mod(VOX[1], 8) + 64 * np.mod(VOX[2], 8))
    b = [tuple(x) for x in c.tolist()].index(blk)
    cand = sc.export_candidates()
    rows = [i for i, k in enumerate(cand["key"].tolist()) if tuple(k[:3]) == blk and k[3] == li]
    assert len(rows) == 1 and not cand["unresolved"][rows[0]]
    states = sorted([(round(F[b, li], 12), int(W[b, li])), (round(cand["F"][rows[0]], 12), int(cand["W"][rows[0]]))])
    assert states == [(0.125, 1), (0.25, 1)]
    # the same pose moved by a tenth of a pixel: no tie, both states take f = 1/4
    T2 = rotated_pose_through(VOX, S2, (0.1251, 0.0625, 1.0))
    img2 = depth_image()
    sc.integrate(img2, K2, T2)
    c, F, W = sc.export()
    cand = sc.export_candidates()
    rows = [i for i, k in enumerate(cand["key"].tolist()) if tuple(k[:3]) == blk and k[3] == li]
    assert len(rows) == 1
    states = sorted([(round(F[b, li], 9), int(W[b, li])), (round(cand["F"][rows[0]], 9), int(cand["W"][rows[0]]))])
    want = sorted([(round((0.125 + 0.25) / 2, 9), 2), (round((0.25 + 0.25) / 2, 9), 2)])
    assert states == want, (states, want)
