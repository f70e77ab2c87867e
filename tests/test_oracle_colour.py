"""Pins of the colour-voxel oracle (section "Framework Flexibility": a voxel may
carry an RGB colour and a colour weight, fused beside the depth).  The paper
gives the voxel type only, so the update is a reading (stated in the oracle):
a voxel whose depth update runs takes the colour at the same pixel when it lies
inside the band (eta <= mu); each channel keeps the running average of its
samples rounded to the nearest integer (ties to even); the colour weight counts
samples up to min(max_w, 255).

Pins: a fronto-parallel plane at 1 m seen head-on, with uniform colour images,
against exact rational arithmetic worked out here -- which voxels take colour
(the band, by each voxel's exact depth), the averages with their ties, the
weight cap -- and the colour read at the plane's raycast hits."""
from fractions import Fraction

import numpy as np

import oracle

W, H = 64, 48
K = (60.0, 60.0, 31.5, 23.5)
S, MU = 0.01, 0.04
T = np.eye(4)


def plane_scene(max_w=100):
    o = oracle.Scene(S, MU, max_w, 1 << 12, 1 << 10)
    o.enable_colour()
    return o


Z0 = 1.005   # the band [0.965, 1.045] starts inside block 12 ([0.96, 1.04)), so the
             # allocated blocks hold voxels in front of the band too


def frame(rgb):
    d = np.full((H, W), Z0, np.float32)
    c = np.zeros((H, W, 4), np.uint8)
    c[..., :3] = rgb
    return d, c


def rhe(q: Fraction) -> int:
    """round half to even"""
    f = q.numerator // q.denominator
    r = q - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return f


def band_masks(coords):
    """per voxel of the exported blocks: strictly inside the band (|eta| < mu by a
    margin), strictly outside in front (eta > mu by a margin), and the voxels the
    depth update reaches (projected inside the border of the image)"""
    b = coords.astype(np.int64)
    l = np.arange(512)
    lx, ly, lz = l % 8, (l // 8) % 8, l // 64
    vx = 8 * b[:, 0:1] + lx[None]
    vy = 8 * b[:, 1:2] + ly[None]
    vz = 8 * b[:, 2:3] + lz[None]
    z = vz * S
    eta = float(np.float32(Z0)) - z
    with np.errstate(divide="ignore", invalid="ignore"):
        x = K[0] * vx * S / z + K[2]
        y = K[1] * vy * S / z + K[3]
    seen = (z > 0) & (x >= 1.01) & (x <= W - 2.01) & (y >= 1.01) & (y <= H - 2.01)
    inside = seen & (np.abs(eta) < MU - 1e-6)
    front = seen & (eta > MU + 1e-6)
    return inside, front


def test_band_voxels_take_the_colour():
    o = plane_scene()
    o.integrate_colour(*frame((200, 100, 50)), K, T)
    coords, F, Wt = o.export()
    C = o.export_colour()
    inside, front = band_masks(coords)
    assert inside.sum() > 1000 and front.sum() > 100
    assert np.all(C[inside][:, :3] == [200, 100, 50]) and np.all(C[inside][:, 3] == 1)
    # in front of the band the depth is updated (F = 1, W = 1) but no colour taken
    assert np.all(Wt[front] == 1) and np.all(C[front] == 0)


def test_running_average_with_ties_to_even_and_the_cap():
    for max_w in (100, 1):
        o = plane_scene(max_w)
        seq = [(200, 100, 50), (53, 100, 0), (0, 255, 3)]
        want = np.array([0, 0, 0]), 0
        c, w = [Fraction(0)] * 3, 0
        for rgb in seq:
            o.integrate_colour(*frame(rgb), K, T)
            c = [Fraction(rhe((w * c[i] + rgb[i]) / Fraction(w + 1))) for i in range(3)]
            w = min(w + 1, max_w, 255)
        coords, _, _ = o.export()
        C = o.export_colour()
        inside, _ = band_masks(coords)
        assert np.all(C[inside][:, :3] == [int(x) for x in c]), (max_w, C[inside][0], c)
        assert np.all(C[inside][:, 3] == w)
    # the tie (200 + 53) / 2 = 126.5 goes to 126 (even), not 127; with max_w = 1
    # the third frame halves: (126 + 0) / 2 = 63
    assert rhe(Fraction(253, 2)) == 126 and rhe(Fraction(251, 2)) == 126


def test_colour_at_the_raycast_hits():
    o = plane_scene()
    o.integrate_colour(*frame((10, 20, 30)), K, T)
    pts = o.raycast(W, H, K, T)[0].astype(np.float32)
    hit = pts[..., 3] > 0
    assert hit.mean() > 0.85
    col = o.colour_at(pts)
    assert np.all(col[~hit] == 0)
    # rays away from the image border meet the plane, whose band took the colour
    # (the border's voxels are never updated: their projections fall outside
    # [1, W - 2] x [1, H - 2])
    inner = np.zeros_like(hit)
    inner[3:-3, 3:-3] = True
    on = hit & inner & (np.abs(pts[..., 2] - Z0) < 0.005)
    assert on.sum() > 0.8 * inner.sum()
    assert np.all(col[on] == [10, 20, 30, 255])
    # a point off the volume reads nothing
    far = np.array([[50.0, 50.0, 50.0, 1.0]], np.float32)
    assert np.all(o.colour_at(far) == 0)


def test_colour_at_reads_the_nearest_voxel():
    """Against the exported voxels, indexed here: the colour at a point is that of
    voxel floor(p / s + 1/2), on a volume whose colours vary from voxel to voxel."""
    import synth
    st = synth.make_stream("tiny", n_frames=3)
    cl = synth.colour_frames(st)
    o = oracle.Scene.from_params(st.params)
    o.enable_colour()
    for f in range(3):
        o.integrate_colour(st.depth[f], cl[f], st.intrinsics, st.T_wc[f])
    coords, _, _ = o.export()
    C = o.export_colour()
    s = st.params["voxel_size"]
    where = {tuple(k): i for i, k in enumerate(coords.tolist())}
    rng = np.random.default_rng(3)
    blk = coords[rng.integers(0, len(coords), 2000)]
    v = blk * 8 + rng.integers(0, 8, (2000, 3))
    p = np.concatenate([(v + rng.uniform(-0.49, 0.49, (2000, 3))) * s, np.ones((2000, 1))], 1).astype(np.float32)
    got = o.colour_at(p)
    vv = np.floor(p[:, :3].astype(np.float64) / s + 0.5).astype(np.int64)
    want = np.zeros((2000, 4), np.uint8)
    for i in range(2000):
        k = tuple((vv[i] // 8).tolist())
        if k in where:
            l = vv[i] - 8 * np.array(k)
            want[i, :3] = C[where[k], l[0] + 8 * l[1] + 64 * l[2], :3]
            want[i, 3] = 255
    assert (want[:, 3] > 0).mean() > 0.9 and len(np.unique(want[:, 0])) > 20
    assert np.array_equal(got, want)
