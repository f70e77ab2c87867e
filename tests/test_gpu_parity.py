"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: the allocated block set is bit-exact; every voxel's weight is bit-exact
and |dF| <= 1e-5 (|dSDF| <= 1e-5 mu) against the oracle's binary64 state, or,
where one of its updates took a decision within the binary32 error bound of a
threshold, against one of the other states the oracle keeps for it
(gpu_util.compare_volumes).  The end-to-end raycast of each side's own volume
is held to fraction bars (gpu_util.compare_raycast); the raycast's per-pixel
parity on identical volumes is in test_gpu_raycast.py."""
import numpy as np
import pytest

from synth import make_stream
from tests.gpu_util import (compare_raycast, compare_volumes, fuse_gpu, fuse_oracle, gpu, K_of,
                            ragged_stream)

pytestmark = pytest.mark.gpu


def test_tiny_f32_per_frame():
    st = make_stream("tiny")
    print("case: tiny f32, 10 frames 160x120", flush=True)
    g, grays, gstats = fuse_gpu(st, ray_frames=(0, 9), per_frame_stats=True)
    o, orays, ostats = fuse_oracle(st, ray_frames=(0, 9), per_frame_stats=True)
    for f, (a, b) in enumerate(zip(gstats, ostats)):
        assert a["n_visible_last"] == b["n_visible"], f
        assert a["n_allocated"] == b["n_allocated"], f
        assert abs(a["n_updated_last"] - b["n_updated_last"]) <= b["n_ambiguous_last"], f
    mx, rms, _ = compare_volumes(g.export(), o.export(), cands=o.export_candidates())
    print(f"max|dF| {mx:.2e} rms {rms:.2e}")
    for f in (0, 9):
        print(compare_raycast(grays[f], orays[f], st.T_wc[f]))


def test_vga_30_frames():
    st = make_stream("vga", n_frames=30)
    print("case: vga f32, 30 frames 640x480, 2^20 buckets", flush=True)
    g, grays, gstats = fuse_gpu(st, ray_frames=(29,))
    o, orays, ostats = fuse_oracle(st, ray_frames=(29,))
    assert g.stats()["n_excess_used"] == o.stats()["n_excess_used"]
    mx, rms, _ = compare_volumes(g.export(), o.export(), cands=o.export_candidates())
    print(f"max|dF| {mx:.2e} rms {rms:.2e}")
    print(compare_raycast(grays[29], orays[29], st.T_wc[29]))


def test_ragged_image_and_invalid_pixels():
    # 97 x 61 image (not a multiple of the 16x16 tile), NaN / inf / negative pixels
    st = ragged_stream()
    print("case: ragged 97x61 with invalid pixels", flush=True)
    g, grays, _ = fuse_gpu(st, ray_frames=(3,))
    o, orays, _ = fuse_oracle(st, ray_frames=(3,))
    compare_volumes(g.export(), o.export(), cands=o.export_candidates())
    print(compare_raycast(grays[3], orays[3], st.T_wc[3], min_cohit=0.99, min_close=0.99))


def test_empty_frame_allocates_nothing():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=1)
    sc = itm.Scene.from_params(st.params)
    z = torch.zeros((st.height, st.width), dtype=torch.float32, device="cuda")
    sc.integrate(z, K_of(st), st.T_wc[0])
    s = sc.stats()
    assert s["n_allocated"] == 0 and s["n_visible_last"] == 0 and s["n_updated_last"] == 0
    p, n = sc.raycast(K_of(st), st.T_wc[0])
    assert float(p.abs().sum()) == 0.0 and float(n.abs().sum()) == 0.0
    coords, F, W = sc.export()
    assert len(coords) == 0


def test_overflow_small_table():
    """A table far too small: the GPU allocates a subset of the oracle's crossed
    blocks, with the same counts (bucket slots, then the excess list, then drops)."""
    import oracle
    st = make_stream("tiny", n_frames=1)
    params = dict(st.params, n_buckets=64, n_excess=8)
    print("case: overflow 64 buckets + 8 excess", flush=True)
    g, _, _ = fuse_gpu(st, params=params)
    o, _, _ = fuse_oracle(st, params=params)
    gs, os_ = g.stats(), o.stats()
    assert gs["n_allocated"] == os_["n_allocated"]
    assert gs["n_excess_used"] == os_["n_excess_used"] == 8
    assert gs["n_dropped_total"] == os_["n_dropped_total"] > 0
    # crossed blocks: the oracle with a table large enough to hold all of them
    big = fuse_oracle(st, params=dict(st.params))[0]
    allc = {tuple(c) for c in big.export(with_values=False)[0].tolist()}
    gc = {tuple(c) for c in g.export(values=False)[0].tolist()}
    assert gc <= allc


def test_repeatable():
    st = make_stream("tiny", n_frames=5)
    a = fuse_gpu(st)[0].export()
    b = fuse_gpu(st)[0].export()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_side_stream():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, _ = fuse_gpu(st)
        out = g.export()
    o, _, _ = fuse_oracle(st)
    compare_volumes(out, o.export(), cands=o.export_candidates())


def test_invalid_arguments():
    itm, torch = gpu()
    with pytest.raises(itm.ItmError):
        itm.Scene(0.01, 0.04, 100, 1000, 16)          # buckets not a power of two
    with pytest.raises(itm.ItmError):
        itm.Scene(0.01, 0.04, 300, 1024, 16, fmt="s16u8")   # weight cap above uint8
    with pytest.raises(itm.ItmError):
        itm.Scene(-0.01, 0.04, 100, 1024, 16)
    sc = itm.Scene(0.01, 0.04, 100, 1024, 16)
    d = torch.zeros((10, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(itm.ItmError):   # image too small for the library
        sc.integrate(torch.zeros((2, 2), dtype=torch.float32, device="cuda"),
                     (100.0, 100.0, 1.0, 1.0, 2, 2), np.eye(4))
    with pytest.raises(ValueError):      # tensor does not match the image size
        sc.integrate(d, (100.0, 100.0, 5.0, 5.0, 12, 10), np.eye(4))
    T = np.eye(4)
    T[0, 3] = np.nan
    with pytest.raises(itm.ItmError):
        sc.integrate(d, (100.0, 100.0, 5.0, 5.0, 10, 10), T)


def test_profile_counts_every_launch():
    """Per-kernel timing: with profiling on, every launch of a frame carries its
    own event pair on its dispatch and is counted once, with a positive time;
    reading resets the counts, and launches with profiling off are not counted."""
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=6)
    print("case: tiny, profiled frames 1..5", flush=True)
    sc = itm.Scene.from_params(st.params)
    sc.set_search_range(True)
    K = K_of(st)
    depth = torch.from_numpy(st.depth).cuda()
    pts = torch.empty((st.height, st.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    sc.integrate(depth[0], K, st.T_wc[0])
    sc.raycast(K, st.T_wc[0], pts, nrm)
    sc.profile(True)
    for f in range(1, 6):
        sc.integrate(depth[f], K, st.T_wc[f])
        sc.raycast(K, st.T_wc[f], pts, nrm)
    sc.profile(False)
    r = sc.profile_read()
    for k in ("alloc", "integrate", "raycast"):
        ms, n = r[k]
        assert n == 5, (k, n)
        assert 0.0 < ms / n < 5.0, (k, ms)
    assert all(r[k][1] == 0 for k in ("refine", "icp_fine", "icp_coarse"))
    sc.integrate(depth[0], K, st.T_wc[0])
    assert all(n == 0 for _, n in sc.profile_read().values())
    sc.close()


def test_out_of_memory_is_a_status():
    """A table the device cannot hold (2^28 buckets: a 2.2 TB voxel block array)
    fails with ITM_ERR_OOM, frees what it had allocated, and leaves the device
    usable."""
    itm, torch = gpu()
    print("case: scene creation beyond HBM", flush=True)
    with pytest.raises(itm.ItmError) as ei:
        itm.Scene(0.01, 0.04, 100, 1 << 28, 1 << 20)
    assert ei.value.status == itm.ITM_ERR_OOM, ei.value
    st = make_stream("tiny", n_frames=2)
    g, _, _ = fuse_gpu(st)
    o, _, _ = fuse_oracle(st)
    compare_volumes(g.export(), o.export(), cands=o.export_candidates())
