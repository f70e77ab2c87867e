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
