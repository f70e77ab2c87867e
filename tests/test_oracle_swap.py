"""Pins of the oracle's swapping schedule (section "Swapping"): a device pool of
voxel blocks smaller than the map, host copies of the blocks that left the view,
and the secondary integration that merges a host copy back into a block that
new frames have fused into meanwhile."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from synth import make_stream


def fuse(orc, st, n, swap=None, params=None):
    sc = orc.Scene.from_params(params or st.params)
    if swap:
        sc.enable_swapping(*swap)
    stats = []
    for f in range(n):
        sc.integrate(st.depth[f], st.intrinsics, st.T_wc[f])
        if swap:
            stats.append(sc.swap_stats())
    return sc, stats


def test_swapping_keeps_the_running_average(orc):
    """Below the weight cap a running average is the mean of all samples, and
    joining two means by their weights is the mean of the union: the swapped
    map (host copies merged, where a copy is still pending, on export) equals
    the map fused without swapping, for any pool and transfer sizes."""
    st = make_stream("vga", n_frames=40)
    params = dict(st.params, max_w=100000)
    ref, _ = fuse(orc, st, 40, params=params)
    rc, rF, rW = ref.export()
    for swap in ((40000, 64, 64), (40000, 4000, 4000), (40000, 7, 3000)):
        sc, stats = fuse(orc, st, 40, swap=swap, params=params)
        c, F, W = sc.export()
        assert np.array_equal(c, rc) and np.array_equal(W, rW)
        assert np.abs(F - rF).max() < 1e-12
        assert sum(s["swapped_out_last"] for s in stats) > 1000      # it did swap
        assert max(s["swapped_in_last"] for s in stats) <= swap[1]
        assert max(s["swapped_out_last"] for s in stats) <= swap[2]
        for s in stats:
            assert s["n_device"] <= swap[0]
        last = stats[-1]
        # every block is on the device or (only) on the host
        assert last["n_device"] + last["n_host_only"] == len(c)
        assert last["no_block_total"] == 0


def test_pool_smaller_than_the_map(orc):
    """A pool of fewer blocks than the map allocates: the device holds the
    blocks in view, the rest live on the host."""
    st = make_stream("vga", n_frames=60)
    sc, stats = fuse(orc, st, 60, swap=(12000, 2000, 4000))
    n = len(sc.export(with_values=False)[0])
    assert n > 12000 and max(s["n_device"] for s in stats) <= 12000
    assert stats[-1]["no_block_total"] == 0
    assert stats[-1]["n_host_only"] > 0


def test_merge_at_the_weight_cap(orc):
    """One voxel on the optical axis at 1 m: frames 1-3 see a plane (W reaches
    max_w = 3), frame 4 sees nothing (the block leaves the view and goes to the
    host), frame 5 sees the plane again (a fresh device block fuses one sample),
    and the host copy merges back: F = (1 f5 + 3 F_h) / 4, W = min(4, 3)."""
    S, MU = 0.01, 0.0625
    K = (10.0, 10.0, 3.5, 3.5)
    W_img = H_img = 8
    sc = orc.Scene(S, MU, 3, 1 << 8, 1 << 6)
    sc.enable_swapping(1000, 1000, 1000)
    depths = [1.03125, 1.015625, 1.0078125, None, 1.046875]
    z_v = Fr(float(np.float32(S))) * 100     # voxel (0, 0, 100)
    samples = []
    for d in depths:
        img = np.zeros((H_img, W_img), np.float32) if d is None else np.full((H_img, W_img), d, np.float32)
        sc.integrate(img, K, np.eye(4))
        if d is not None:
            samples.append(min(Fr(1), (Fr(d) - z_v) / Fr(MU)))
    st = sc.swap_stats()
    assert st["swapped_out_total"] >= 1 and st["swapped_in_total"] >= 1 and st["n_pending"] == 0
    c, F, W = sc.export()
    b = [tuple(x) for x in c.tolist()].index((0, 0, 12))
    li = 0 + 8 * 0 + 64 * (100 - 96)
    # the running average of the first three (the third update at W = 2 -> 3)
    Fh = (samples[0] + samples[1] + samples[2]) / 3
    want = (1 * samples[3] + 3 * Fh) / 4
    assert W[b, li] == 3
    assert abs(F[b, li] - float(want)) < 1e-12
