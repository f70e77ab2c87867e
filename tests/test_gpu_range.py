"""Expected depth ranges (section "Raycast", the search range) on the GPU through
the C ABI against the oracle.

Bars: the range image is bit-exact (both sides form the block boxes in binary64
in one fixed order and round outwards to binary32), whichever way the GPU bins
the rectangles -- during the integration at the frame's own pose, afterwards at
another pose, or in the exact fallback for a tile whose bin overflowed.  The
raycast inside the ranges meets the same bars as the fixed-range raycast
(gpu_util.compare_raycast) against the oracle's raycast inside the oracle's
ranges."""
import numpy as np
import pytest

from synth import make_stream
from tests.gpu_util import compare_raycast, fuse_gpu, fuse_oracle, gpu, K_of, ragged_stream

pytestmark = pytest.mark.gpu


def _same(a, b):
    """Bit equality of two float32 range images."""
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


def _ranges(g, o, st, T):
    got = g.expected_depths(K_of(st), T).cpu().numpy()
    want = o.expected_depths(st.width, st.height, st.intrinsics, T)
    return got, want


@pytest.mark.parametrize("search_range", [False, True])
def test_tiny_range_image(search_range):
    st = make_stream("tiny")
    print(f"case: tiny range image, bins during integration {search_range}", flush=True)
    g, _, _ = fuse_gpu(st, search_range=search_range)
    o, _, _ = fuse_oracle(st)
    for f in (9, 0, 5):       # own pose (reuses the frame's bins when on), then other poses
        got, want = _ranges(g, o, st, st.T_wc[f])
        covered = want[..., 0] <= want[..., 1]
        assert covered.mean() > 0.5
        assert _same(got, want), f"frame {f}: {np.count_nonzero(got != want)} values differ"


def test_vga_range_image_and_other_pose():
    st = make_stream("vga", n_frames=30)
    print("case: vga 30 frames, range image at own and other poses", flush=True)
    g, _, _ = fuse_gpu(st, search_range=True)
    o, _, _ = fuse_oracle(st)
    for f in (29, 20):
        got, want = _ranges(g, o, st, st.T_wc[f])
        assert _same(got, want), f"frame {f}: {np.count_nonzero(got != want)} values differ"


def test_ragged_range_image():
    st = ragged_stream()
    print("case: ragged 97x61 range image", flush=True)
    g, _, _ = fuse_gpu(st, search_range=True)
    o, _, _ = fuse_oracle(st)
    got, want = _ranges(g, o, st, st.T_wc[3])
    assert _same(got, want)


@pytest.mark.parametrize("cap", [1, 3])
def test_overflowing_bins_stay_exact(cap):
    """With room for 1 or 3 rectangles per tile nearly every tile overflows and
    takes the exact fallback."""
    st = make_stream("tiny", n_frames=4)
    print(f"case: tiny, tile capacity {cap}", flush=True)
    g, _, _ = fuse_gpu(st, search_range=True, tile_capacity=cap)
    o, _, _ = fuse_oracle(st, frames=4)
    for f in (3, 1):
        got, want = _ranges(g, o, st, st.T_wc[f])
        assert _same(got, want)


def test_tiny_ranged_raycast():
    st = make_stream("tiny")
    print("case: tiny ranged raycast", flush=True)
    g, grays, _ = fuse_gpu(st, ray_frames=(0, 9), search_range=True)
    o, orays, _ = fuse_oracle(st, ray_frames=(0, 9), search_range=True)
    for f in (0, 9):
        print(compare_raycast(grays[f], orays[f], st.T_wc[f]))


def test_vga_ranged_raycast():
    st = make_stream("vga", n_frames=30)
    print("case: vga 30 frames ranged raycast", flush=True)
    g, grays, _ = fuse_gpu(st, ray_frames=(29,), search_range=True)
    o, orays, _ = fuse_oracle(st, ray_frames=(29,), search_range=True)
    print(compare_raycast(grays[29], orays[29], st.T_wc[29]))
    # a pixel outside every range is a miss on both sides
    zr = o.expected_depths(st.width, st.height, st.intrinsics, st.T_wc[29])
    empty = ~(zr[..., 0] <= zr[..., 1])
    assert not (grays[29][0][..., 3] > 0)[empty].any()


def test_ranged_raycast_at_other_pose_and_overflow():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=6)
    g, _, _ = fuse_gpu(st, search_range=True, tile_capacity=2)
    o, _, _ = fuse_oracle(st, frames=6)
    T = st.T_wc[2]
    p, n = g.raycast(K_of(st), T)
    zr = o.expected_depths(st.width, st.height, st.intrinsics, T)
    want = o.raycast(st.width, st.height, st.intrinsics, T, zrange=zr)
    print(compare_raycast((p.cpu().numpy(), n.cpu().numpy()), want, T))


def test_range_without_frames_and_toggling():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=3)
    sc = itm.Scene.from_params(st.params)
    sc.set_search_range(True)
    K = K_of(st)
    zr = sc.expected_depths(K, st.T_wc[0]).cpu().numpy()
    assert np.all(np.isinf(zr[..., 0])) and np.all(zr[..., 1] == 0)
    p, n = sc.raycast(K, st.T_wc[0])
    assert float(p.abs().sum()) == 0.0      # nothing visible: every pixel misses
    # off for one frame, on again: the bins are rebuilt, results still exact
    sc.set_search_range(False)
    sc.integrate(torch.from_numpy(st.depth[0]).cuda(), K, st.T_wc[0])
    sc.set_search_range(True)
    sc.integrate(torch.from_numpy(st.depth[1]).cuda(), K, st.T_wc[1])
    o, _, _ = fuse_oracle(st, frames=2)
    got = sc.expected_depths(K, st.T_wc[1]).cpu().numpy()
    assert _same(got, o.expected_depths(st.width, st.height, st.intrinsics, st.T_wc[1]))
    with pytest.raises(itm.ItmError):
        sc.set_search_range(True, 1 << 20)


def test_blocks_listed_when_the_workgroup_set_is_full():
    """A band far deeper than a block (voxel 3 mm, mu 0.5 m) makes a 16x16 tile's
    pixels cross more distinct blocks (up to ~4200) than the allocation
    kernel's per-workgroup set holds (2048): those blocks are listed, and their
    rectangles binned, one by one.  Block set, visible count and the range image
    at the frame's own pose (bins filled during allocation, room for every
    rectangle) must still equal the oracle's."""
    import oracle
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=1)
    params = dict(voxel_size=0.003, mu=0.5, max_w=100, n_buckets=2 ** 18, n_excess=2 ** 17)
    print("case: tiny frame 0, voxel 3 mm, mu 0.5 m (workgroup sets overflow)", flush=True)
    g = itm.Scene.from_params(params)
    g.set_search_range(True, 8192)
    g.integrate(torch.from_numpy(np.ascontiguousarray(st.depth[0])).cuda(), K_of(st), st.T_wc[0])
    o = oracle.Scene.from_params(params)
    n_vis = o.allocate(st.depth[0], st.intrinsics, st.T_wc[0])
    assert g.stats()["n_visible_last"] == n_vis and g.stats()["n_allocated"] == o.stats()["n_allocated"]
    gc = g.export(values=False)[0]
    oc = o.export(with_values=False)[0]
    assert np.array_equal(gc, oc)
    got, want = _ranges(g, o, st, st.T_wc[0])
    assert _same(got, want), f"{np.count_nonzero(got != want)} values differ"
    g.close()
