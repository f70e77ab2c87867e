"""Pins of the oracle's expected depth range (section "Raycast", the search range
rendered from the visible blocks) and of the raycast that searches inside it.

* a single visible block seen head-on: the covered pixels and the depth range are
  worked out by hand below;
* on the tiny stream, every pixel whose ray passes through a visible block's box
  (exact slab intersection, written independently here) is covered, with the
  entry and exit depths inside its range;
* the raycast inside the range finds the same surface as the fixed-range raycast
  wherever that one hits a visible block.
"""
import numpy as np
import pytest

from synth import make_stream


def test_single_block_by_hand(orc):
    """One valid pixel (53, 53) at depth 1.0 m, identity pose, f = 100, c = 50,
    s = 1 cm, mu = 2 cm.  The band z in [0.98, 1.02] along the ray (0.03, 0.03, 1)
    lies in block (0, 0, 12) (block edge 8 cm: z 0.96..1.04), the only visible one.
    Its box [8k - 1/2, 8k + 7 1/2] s is x, y in [-0.005, 0.075], z in [0.955, 1.035];
    projected: x in [100 (-0.005 / 0.955) + 50, 100 (0.075 / 0.955) + 50] =
    [49.476, 57.853], so pixels 50..57 on both axes."""
    W = H = 100
    K = np.array([100.0, 100.0, 50.0, 50.0])
    depth = np.zeros((H, W), np.float32)
    depth[53, 53] = 1.0
    sc = orc.Scene(0.01, 0.02, 100, 2 ** 12, 2 ** 10)
    sc.integrate(depth, K, np.eye(4))
    assert sc.visible_keys().tolist() == [[0, 0, 12]]
    zr = sc.expected_depths(W, H, K, np.eye(4))
    covered = zr[..., 0] <= zr[..., 1]
    want = np.zeros((H, W), bool)
    want[50:58, 50:58] = True
    assert np.array_equal(covered, want)
    assert np.all(np.isinf(zr[~want][:, 0])) and np.all(zr[~want][:, 1] == 0)
    zmin, zmax = zr[50:58, 50:58, 0], zr[50:58, 50:58, 1]
    # the faces at 95.5 s and 103.5 s (s = 0.01 as binary32), rounded outwards
    s32 = float(np.float32(0.01))
    near, far = 95.5 * s32, 103.5 * s32
    assert abs(near - 0.955) < 1e-7 and abs(far - 1.035) < 1e-7
    assert np.all(zmin == zmin[0, 0]) and np.all(zmax == zmax[0, 0])
    assert float(zmin[0, 0]) <= near < float(np.nextafter(zmin[0, 0], np.float32(2)))
    assert float(np.nextafter(zmax[0, 0], np.float32(0))) < far <= float(zmax[0, 0])


def test_block_behind_camera_covers_image(orc):
    """A visible block that straddles the camera plane cannot be projected; it
    covers the whole image from depth 0."""
    W = H = 40
    K = np.array([40.0, 40.0, 20.0, 20.0])
    depth = np.zeros((H, W), np.float32)
    depth[20, 20] = 0.05         # band [0.03, 0.07]: block z index 0, box z from -0.005
    sc = orc.Scene(0.01, 0.02, 100, 2 ** 12, 2 ** 10)
    sc.integrate(depth, K, np.eye(4))
    keys = sc.visible_keys()
    assert len(keys) >= 1 and np.all(keys[:, 2] == 0)
    zr = sc.expected_depths(W, H, K, np.eye(4))
    assert np.all(zr[..., 0] == 0.0)
    assert np.all(zr[..., 1] >= np.float32(0.075))


def _slab(o, d, lo, hi):
    """Entry and exit ray parameters of the box [lo, hi] (None if missed)."""
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return None
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t0 <= t1 and t1 > 0 else None


@pytest.fixture(scope="module")
def tiny_scene(orc):
    st = make_stream("tiny")
    sc = orc.fuse_stream(st)
    return st, sc


def test_range_contains_every_block_crossing(tiny_scene):
    st, sc = tiny_scene
    W, H, (fx, fy, cx, cy) = st.width, st.height, st.intrinsics
    T = st.T_wc[-1]
    zr = sc.expected_depths(W, H, st.intrinsics, T).astype(np.float64)
    keys = sc.visible_keys()
    s = st.params["voxel_size"]
    R, t = T[:3, :3], T[:3, 3]
    rng = np.random.default_rng(5)
    pix = rng.integers(0, [W, H], size=(400, 2))
    checked = 0
    for u, v in pix:
        dc = np.array([(u - cx) / fx, (v - cy) / fy, 1.0])   # camera ray, z component 1
        dw = R @ dc
        for k in keys:
            lo = (8.0 * k - 0.5) * s
            hi = (8.0 * k + 7.5) * s
            hit = _slab(t, dw, lo, hi)
            if hit is None:
                continue
            # parameter along dw is the camera depth (dc has z = 1)
            z0, z1 = max(hit[0], 0.0), hit[1]
            assert zr[v, u, 0] <= z0 + 1e-9 and z1 - 1e-9 <= zr[v, u, 1], (u, v, k)
            checked += 1
    assert checked > 100


def test_range_is_tight_for_fronto_parallel_block(orc):
    """Not merely conservative: for a block straight ahead, the pixel at the
    optical axis gets exactly the box's nearest and farthest face depths."""
    W = H = 100
    K = np.array([100.0, 100.0, 49.5, 49.5])   # axis between pixels 49 and 50
    depth = np.zeros((H, W), np.float32)
    depth[50, 50] = 1.0
    sc = orc.Scene(0.01, 0.02, 100, 2 ** 12, 2 ** 10)
    sc.integrate(depth, K, np.eye(4))
    zr = sc.expected_depths(W, H, K, np.eye(4))
    assert abs(float(zr[50, 50, 0]) - 0.955) < 1e-7
    assert abs(float(zr[50, 50, 1]) - 1.035) < 1e-7


def test_ranged_raycast_matches_fixed_range(tiny_scene):
    st, sc = tiny_scene
    W, H = st.width, st.height
    T = st.T_wc[-1]
    zr = sc.expected_depths(W, H, st.intrinsics, T)
    p0, n0, z0, _, s0 = sc.raycast(W, H, st.intrinsics, T)
    p1, n1, z1, _, s1 = sc.raycast(W, H, st.intrinsics, T, zrange=zr)
    # hits outside every range are impossible; hits of the fixed-range march that
    # lie in a visible block are found again, at the same depth
    covered = zr[..., 0] <= zr[..., 1]
    assert np.all(~(z1 > 0) | covered)
    s = st.params["voxel_size"]
    vis = {tuple(k) for k in sc.visible_keys().tolist()}
    blk = np.floor(p0[..., :3] / s + 0.5).astype(np.int64) // 8
    in_vis = np.array([tuple(b) in vis for b in blk.reshape(-1, 3)]).reshape(H, W) & (z0 > 0)
    assert in_vis.mean() > 0.9
    both = in_vis & (z1 > 0)
    assert both.sum() >= 0.99 * in_vis.sum()
    # A march that starts elsewhere samples the noisy far plane at other points
    # and can settle on a neighbouring zero crossing (measured: 97.7% of co-hits
    # within 1 mm, the rest 1-3 cm apart, as many nearer as farther).  Against
    # the dense zero-crossing search both marches do equally well.
    assert (np.abs(z1 - z0)[both] < 1e-3).mean() > 0.97
    zx = sc.raycast_crossing(W, H, st.intrinsics, T)
    agree0 = (np.abs(z0 - zx)[both] < 1e-3).mean()
    agree1 = (np.abs(z1 - zx)[both] < 1e-3).mean()
    assert agree1 >= agree0 - 0.005
    # the range saves march steps (measured 26.8 -> 10.3 per ray)
    assert s1[both].mean() < 0.6 * s0[both].mean()
    print(f"mean steps fixed {s0[both].mean():.2f}, ranged {s1[both].mean():.2f}; "
          f"zero-crossing agreement {agree0:.4f} / {agree1:.4f}")


def test_plane_raycast_in_range_closed_form(orc):
    """The fused fronto-parallel plane z = Z0, raycast inside its expected
    ranges: every inner pixel hits at camera depth Z0 up to the two-step
    refinement residual 2 s (1 - cos(theta))^2 (the bound of the fixed-range
    march, which the same surface samples obey wherever the march starts)."""
    from tests.test_oracle_scene import _plane_stream
    Z0, s, mu = 1.3, 0.01, 0.04
    depth, T, K = _plane_stream(Z0)
    sc = orc.Scene(s, mu, 100, 2 ** 14, 2 ** 12)
    for f in range(len(depth)):
        sc.integrate(depth[f], K, T[f])
    H, W = depth.shape[1:]
    zr = sc.expected_depths(W, H, K, T[0])
    pts, nrm, zc, fl, st = sc.raycast(W, H, K, T[0], zrange=zr)
    inner = np.zeros((H, W), bool)
    inner[4:-4, 4:-4] = True
    assert (pts[..., 3] > 0)[inner].all()
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    cos_t = 1.0 / np.sqrt(((u - K[2]) / K[0]) ** 2 + ((v - K[3]) / K[1]) ** 2 + 1.0)
    bound = 2 * s * (1 - cos_t) ** 2 + 1e-9
    err = np.abs(zc - float(np.float32(Z0)))
    assert np.all(err[inner] <= bound[inner])
    # the range starts in front of the band [Z0 - mu, Z0 + mu], at most one block
    # edge plus half a voxel before it, so the march enters from the front
    assert np.all(zr[inner][:, 0] >= Z0 - mu - 8.5 * s - 1e-6)
    assert np.all(zr[inner][:, 0] < Z0 - mu)


def test_range_bounds_are_obeyed(orc):
    """A range of (0.25, 4.0) everywhere reproduces the fixed-range raycast over
    [0.25, 4.0] exactly; a range that ends before the plane, or starts behind it,
    finds nothing."""
    from tests.test_oracle_scene import _plane_stream
    Z0, s, mu = 1.3, 0.01, 0.04
    depth, T, K = _plane_stream(Z0)
    sc = orc.Scene(s, mu, 100, 2 ** 14, 2 ** 12)
    for f in range(len(depth)):
        sc.integrate(depth[f], K, T[f])
    H, W = depth.shape[1:]
    full = np.empty((H, W, 2), np.float32)
    full[..., 0], full[..., 1] = 0.25, 4.0         # inside the default [0.2, 5.0]
    b = sc.raycast(W, H, K, T[0], zrange=full)
    sc.set_range(0.25, 4.0)
    a = sc.raycast(W, H, K, T[0])
    sc.set_range(0.2, 5.0)
    assert (a[0][..., 3] > 0).sum() > 10000
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    short = full.copy()
    short[..., 1] = Z0 - 0.06
    assert not (sc.raycast(W, H, K, T[0], zrange=short)[0][..., 3] > 0).any()
    late = full.copy()
    late[..., 0] = Z0 + 0.2
    assert not (sc.raycast(W, H, K, T[0], zrange=late)[0][..., 3] > 0).any()


def test_raycast_reads_about_the_visible_blocks(orc):
    """The benchmark prices a raycast's voxel reads by the frame's visible blocks
    (512 F values and a bucket record each).  Counting what the oracle's ranged
    raycast at the frame's pose actually reads, on the VGA stream: the distinct
    blocks are within 5% of the visible ones, the buckets probed about 1.5x."""
    from synth import make_stream
    st = make_stream("vga", n_frames=20)
    sc = orc.Scene.from_params(st.params)
    for f in range(20):
        sc.integrate(st.depth[f], st.intrinsics, st.T_wc[f])
    args = (st.width, st.height, st.intrinsics, st.T_wc[19])
    blocks, buckets = sc.raycast_touched(*args, zrange=sc.expected_depths(*args))
    vis = sc.stats()["n_visible"]
    print(f"visible {vis}, blocks read {blocks}, buckets probed {buckets}")
    assert abs(blocks - vis) <= 0.05 * vis
    assert vis <= buckets <= 2 * vis
