"""GPU parity of the colour voxels (section "Framework Flexibility": a voxel may
carry a colour and a colour weight; section "Integration": the colour is fused
beside the depth).  The colour update is exact integer arithmetic, so the stored
colours must match the oracle's bit for bit, in every voxel format, jointly with
the voxel's F and W: the oracle's binary64 state, or one of the other states it
keeps where a decision (the band, the pixel) lay within its binary32 error bound; the raycast's colour is the colour
of the hit point's nearest voxel, checked against the oracle's read at the
GPU's own hit points."""
import numpy as np
import pytest

from synth import colour_frames, make_stream
from tests.gpu_util import K_of, compare_volumes, gpu, ragged_stream

pytestmark = pytest.mark.gpu


def fuse_both(st, n, fmt="f32", plain_first=0, params=None):
    """the first `plain_first` frames without colour, the rest with it, on the
    GPU and in the oracle"""
    import oracle
    itm, torch = gpu()
    params = params or st.params
    rgb = colour_frames(st, range(n))
    g = itm.Scene.from_params(params, fmt=fmt)
    o = oracle.Scene.from_params(params)
    g.enable_colour()
    o.enable_colour()
    K = K_of(st)
    depth = torch.from_numpy(np.ascontiguousarray(st.depth[:n])).cuda()
    crgb = torch.from_numpy(rgb).cuda()
    for f in range(n):
        if f < plain_first:
            g.integrate(depth[f], K, st.T_wc[f])
            o.integrate(st.depth[f], st.intrinsics, st.T_wc[f])
        else:
            g.integrate_colour(depth[f], crgb[f], K, st.T_wc[f])
            o.integrate_colour(st.depth[f], rgb[f], st.intrinsics, st.T_wc[f])
    torch.cuda.synchronize()
    return g, o


def check_colours(g, o, fmt="f32"):
    """F, W and colour of every voxel jointly against the oracle's states; the
    compact forms compare colour and weight only (F is quantised)"""
    gc = g.export_colour()
    oc = o.export_colour()
    tol = 1e-5 if fmt == "f32" else 2.0
    compare_volumes(g.export(), o.export(), tol=tol, cands=o.export_candidates(), g_colour=gc, o_colour=oc)
    return gc


def test_tiny_colour_bit_exact():
    st = make_stream("tiny")
    print("colour: tiny, f32, all frames", flush=True)
    g, o = fuse_both(st, st.n_frames)
    gc = check_colours(g, o)
    assert (gc[..., 3] > 0).sum() > 10000           # the band took colour
    assert gc[..., 3].max() == min(st.params["max_w"], 255, st.n_frames)
    g.close()


@pytest.mark.parametrize("fmt", ["f16", "s16u8"])
def test_colour_bit_exact_in_compact_formats(fmt):
    # the colour decision does not depend on how F and W are stored
    st = make_stream("tiny", n_frames=6)
    params = dict(st.params, max_w=min(st.params["max_w"], 255))
    print(f"colour: tiny, {fmt}", flush=True)
    g, o = fuse_both(st, 6, fmt=fmt, params=params)
    check_colours(g, o, fmt)
    g.close()


def test_vga_colour_bit_exact():
    st = make_stream("vga", n_frames=10)
    print("colour: vga, 10 frames", flush=True)
    g, o = fuse_both(st, 10)
    check_colours(g, o)
    g.close()


def test_colour_enabled_after_plain_frames():
    # blocks fused before the first colour frame keep colour weight 0 until a
    # colour sample reaches them; plain frames leave colours as they are
    st = make_stream("tiny", n_frames=8)
    print("colour: plain frames first", flush=True)
    g, o = fuse_both(st, 8, plain_first=4)
    gc = check_colours(g, o)
    assert gc[..., 3].max() == 4
    g.close()


def test_ragged_colour_and_invalid_pixels():
    st = ragged_stream()
    print("colour: ragged 97 x 61", flush=True)
    g, o = fuse_both(st, st.n_frames)
    check_colours(g, o)
    g.close()


@pytest.mark.parametrize("search_range", [False, True])
def test_raycast_colour_matches_nearest_voxel(search_range):
    itm, torch = gpu()
    st = make_stream("vga", n_frames=10)
    print(f"colour raycast: vga, search range {search_range}", flush=True)
    g, o = fuse_both(st, 10)
    if search_range:
        g.set_search_range(True)
        g.integrate_colour(torch.from_numpy(np.ascontiguousarray(st.depth[9])).cuda(),
                           torch.from_numpy(colour_frames(st, [9])[0]).cuda(), K_of(st), st.T_wc[9])
        o.integrate_colour(st.depth[9], colour_frames(st, [9])[0], st.intrinsics, st.T_wc[9])
    K = K_of(st)
    T = st.T_wc[9]
    p0, n0 = g.raycast(K, T)
    p, n, c = g.raycast_colour(K, T)
    torch.cuda.synchronize()
    P, N, Cg = p.cpu().numpy(), n.cpu().numpy(), c.cpu().numpy()
    # points and normals are those of the plain raycast, bit for bit
    assert np.array_equal(P, p0.cpu().numpy()) and np.array_equal(N, n0.cpu().numpy())
    hit = P[..., 3] > 0
    assert hit.mean() > 0.5
    assert np.all(Cg[~hit] == 0)
    Co = o.colour_at(P)
    same = np.all(Cg == Co, axis=-1)
    assert same.mean() >= 0.999, f"colour reads agree at {same.mean():.5f} of pixels"
    # most hits read a voxel that has taken colour
    assert (Cg[hit][:, :3].max(-1) > 0).mean() > 0.95
    g.close()


def test_colour_calls_need_colour_enabled():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=1)
    sc = itm.Scene.from_params(st.params)
    K = K_of(st)
    d = torch.from_numpy(np.ascontiguousarray(st.depth[0])).cuda()
    rgb = torch.zeros((st.height, st.width, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(itm.ItmError):
        sc.integrate_colour(d, rgb, K, st.T_wc[0])
    with pytest.raises(itm.ItmError):
        sc.raycast_colour(K, st.T_wc[0])
    with pytest.raises(itm.ItmError):
        sc.export_colour()
    sc.enable_colour()
    sc.enable_colour()                      # a no-op the second time
    with pytest.raises(ValueError):         # wrong image size, caught by the binding
        sc.integrate_colour(d, rgb[:-1], K, st.T_wc[0])
    sc.integrate_colour(d, rgb, K, st.T_wc[0])
    torch.cuda.synchronize()
    c = sc.export_colour()
    assert c.shape[0] == sc.export(values=False)[0].shape[0]
    assert np.all(c[..., :3] == 0)          # black samples
    sc.close()
