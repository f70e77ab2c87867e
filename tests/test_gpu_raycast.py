"""Raycast parity per pixel (section "Raycast") on identical volumes.

A volume fused by the oracle is quantised to a storage form and loaded into both
a GPU scene (itm_import_blocks, through the C ABI) and a second oracle scene, so
the two march through the same F values.  Every pixel of the GPU raycast must
then match one of the oracle's correct outcomes for that ray
(gpu_util.compare_raycast_exact): the binary64 march's, or another one the
oracle reaches where a sample lay within the binary32 error bound of a rounding
boundary -- both a miss, or both a hit within 0.5 mm of camera depth with the
normal within 8 degrees.  Pixels whose march branched more often than the oracle
follows are counted and reported, not compared."""
import numpy as np
import pytest

import oracle
from synth import make_stream, pose_look_at
from tests.gpu_util import K_of, compare_raycast_exact, gpu, ragged_stream

pytestmark = pytest.mark.gpu

FMTS = ["f32", "f16", "s16u8"]


def quantise(F, fmt):
    """F as the storage form holds it, in binary64 (round to nearest even)"""
    if fmt == "f32":
        return F.astype(np.float32).astype(np.float64)
    if fmt == "f16":
        return F.astype(np.float16).astype(np.float64)
    return np.clip(np.rint(F * 32767.0), -32767, 32767) / 32767.0


def fused_oracle_volume(st, n):
    o = oracle.Scene.from_params(st.params)
    for f in range(n):
        o.integrate(st.depth[f], st.intrinsics, st.T_wc[f])
    return o.export()


def load_both(st, vol, fmt, params=None):
    itm, torch = gpu()
    params = params or st.params
    c, F, W = vol
    Fq = quantise(F, fmt)
    o = oracle.Scene.from_params(params)
    assert o.import_blocks(c, Fq, W) == len(c)
    g = itm.Scene.from_params(params, fmt=fmt)
    g.import_blocks(c, Fq.astype(np.float32), W.astype(np.float32))
    gs = g.stats()
    assert gs["n_allocated"] == len(c) and gs["n_visible_last"] == len(c)
    return g, o


def ray_both(g, o, st, T, search_range):
    itm, torch = gpu()
    K = K_of(st)
    g.set_search_range(search_range)
    p, n = g.raycast(K, T)
    torch.cuda.synchronize()
    args = (st.width, st.height, st.intrinsics, T)
    zr = o.expected_depths(*args) if search_range else None
    return (p.cpu().numpy(), n.cpu().numpy()), o.raycast(*args, zrange=zr, alternatives=True)


def check(g, o, st, poses, search_range):
    out = []
    for T in poses:
        gr, orr = ray_both(g, o, st, T, search_range)
        info = compare_raycast_exact(gr, orr, T)
        assert info["hits"] > 0.3 * info["pixels"]
        assert info["unresolved"] <= 0.005 * info["pixels"]
        out.append(info)
    return out


@pytest.fixture(scope="module")
def tiny_vol():
    st = make_stream("tiny")
    return st, fused_oracle_volume(st, st.n_frames)


@pytest.fixture(scope="module")
def vga_vol():
    st = make_stream("vga", n_frames=30)
    return st, fused_oracle_volume(st, 30)


@pytest.mark.parametrize("search_range", [False, True])
@pytest.mark.parametrize("fmt", FMTS)
def test_tiny(tiny_vol, fmt, search_range):
    st, vol = tiny_vol
    print(f"case: raycast tiny {fmt}, search range {search_range}", flush=True)
    g, o = load_both(st, vol, fmt)
    # the stream's first and last poses and one the stream never took
    other = pose_look_at((0.15, -0.1, -0.05), (0.0, 0.0, 1.2), (0, -1, 0))
    check(g, o, st, [st.T_wc[0], st.T_wc[-1], other], search_range)
    g.close()


@pytest.mark.parametrize("search_range", [False, True])
@pytest.mark.parametrize("fmt", FMTS)
def test_vga(vga_vol, fmt, search_range):
    st, vol = vga_vol
    print(f"case: raycast vga {fmt}, search range {search_range}", flush=True)
    g, o = load_both(st, vol, fmt)
    T = st.T_wc[29].copy()
    T2 = T.copy()
    T2[:3, 3] += np.array([0.03, -0.02, 0.04])
    check(g, o, st, [T, T2], search_range)
    g.close()


@pytest.mark.parametrize("search_range", [False, True])
def test_ragged(search_range):
    st = ragged_stream()
    print(f"case: raycast ragged 97x61, search range {search_range}", flush=True)
    vol = fused_oracle_volume(st, st.n_frames)
    g, o = load_both(st, vol, "f32")
    check(g, o, st, [st.T_wc[0], st.T_wc[3]], search_range)
    g.close()


def test_import_round_trip():
    """export(import(x)) = x on the GPU in every form (values representable in
    the form); the loaded set is the visible set; bad input is refused and
    changes nothing"""
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=3)
    c, F, W = fused_oracle_volume(st, 3)
    for fmt in FMTS:
        Fq = quantise(F, fmt).astype(np.float32)
        g = itm.Scene.from_params(st.params, fmt=fmt)
        g.import_blocks(c, Fq, W.astype(np.float32))
        c2, F2, W2 = g.export()
        assert np.array_equal(c2, c) and np.array_equal(W2, W.astype(np.float32))
        assert np.abs(F2.astype(np.float64) - Fq).max() <= (0 if fmt != "s16u8" else 1e-7)
        bad = W.astype(np.float32).copy()
        bad[0, 0] = st.params["max_w"] + 1
        with pytest.raises(itm.ItmError):
            g.import_blocks(c, Fq, bad)
        with pytest.raises(itm.ItmError):          # a repeated key
            g.import_blocks(np.concatenate([c[:2], c[:1]]), Fq[:3], W[:3].astype(np.float32))
        assert g.stats()["n_allocated"] == len(c)
        g.close()
