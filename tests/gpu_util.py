"""Helpers shared by the GPU parity tests: run a seeded stream through the HIP
library and through the oracle, and compare."""
import numpy as np

SDF_TOL = 1e-5          # |dF| (F = SDF / mu), i.e. |dSDF| <= 1e-5 mu
DEPTH_TOL = 5e-4        # metres, raycast camera depth on co-hit pixels


def gpu():
    import torch
    import paper_1410_0925_amd as itm
    if not __import__("os").path.exists(itm.LIB_PATH):
        from paper_1410_0925_amd import build
        build.build()
    assert torch.cuda.is_available()
    return itm, torch


def K_of(stream):
    return tuple(stream.intrinsics) + (stream.width, stream.height)


def fuse_gpu(stream, frames=None, fmt="f32", params=None, ray_frames=(), per_frame_stats=False,
             search_range=False, tile_capacity=0):
    itm, torch = gpu()
    n = stream.n_frames if frames is None else frames
    sc = itm.Scene.from_params(params or stream.params, fmt=fmt)
    if search_range:
        sc.set_search_range(True, tile_capacity)
    depth = torch.from_numpy(np.ascontiguousarray(stream.depth[:n])).cuda()
    K = K_of(stream)
    rays, stats = {}, []
    for f in range(n):
        sc.integrate(depth[f], K, stream.T_wc[f])
        if per_frame_stats:
            stats.append(sc.stats())
        if f in ray_frames:
            p, q = sc.raycast(K, stream.T_wc[f])
            rays[f] = (p.cpu().numpy(), q.cpu().numpy())
    torch.cuda.synchronize()
    return sc, rays, stats


def fuse_oracle(stream, frames=None, params=None, ray_frames=(), per_frame_stats=False, search_range=False):
    import oracle
    n = stream.n_frames if frames is None else frames
    sc = oracle.Scene.from_params(params or stream.params)
    rays, stats = {}, []
    for f in range(n):
        sc.integrate(stream.depth[f], stream.intrinsics, stream.T_wc[f])
        if per_frame_stats:
            stats.append(sc.stats())
        if f in ray_frames:
            args = (stream.width, stream.height, stream.intrinsics, stream.T_wc[f])
            zr = sc.expected_depths(*args) if search_range else None
            rays[f] = sc.raycast(*args, zrange=zr)
    return sc, rays, stats


def compare_volumes(g_export, o_export, tol=SDF_TOL):
    gc, gF, gW = g_export
    oc, oF, oW = o_export
    assert gc.shape == oc.shape, (gc.shape, oc.shape)
    assert np.array_equal(gc, oc), "allocated block sets differ"
    assert np.array_equal(gW.astype(np.int64), oW.astype(np.int64)), \
        f"weights differ at {np.count_nonzero(gW != oW)} voxels"
    err = np.abs(gF.astype(np.float64) - oF)
    assert err.max() <= tol, f"max |dF| {err.max():.3e} > {tol}"
    return float(err.max()), float(np.sqrt(np.mean(err[oW > 0] ** 2))) if (oW > 0).any() else 0.0


def ragged_stream():
    """4 frames of a 97 x 61 image (not a multiple of the 16 x 16 tile) of a
    sphere before a plane, with NaN / inf / negative / zero pixels."""
    from synth import Scene as SynthScene, pose_look_at, render_depth
    rng = np.random.default_rng(3)
    K = (80.0, 80.0, 48.3, 30.1)
    scene = SynthScene(spheres=np.array([[0.1, -0.05, 1.0, 0.25]]),
                       planes=np.array([[0.0, 0.0, -1.0, -1.6]]))
    frames, poses = [], []
    for a in np.linspace(-0.1, 0.1, 4):
        T = pose_look_at((a, 0.02, 0.0), (0.1, -0.05, 1.0), (0, -1, 0))
        d = render_depth(scene, K, 97, 61, T).astype(np.float32)
        d += (rng.standard_normal(d.shape) * 0.001).astype(np.float32)
        bad = rng.random(d.shape)
        d[bad < 0.02] = np.nan
        d[(bad >= 0.02) & (bad < 0.03)] = np.inf
        d[(bad >= 0.03) & (bad < 0.04)] = -1.0
        d[(bad >= 0.04) & (bad < 0.05)] = 0.0
        frames.append(d)
        poses.append(T)

    class S:  # minimal stream object
        pass
    st = S()
    st.depth, st.T_wc = np.stack(frames), np.stack(poses)
    st.intrinsics, st.width, st.height = K, 97, 61
    st.n_frames = 4
    st.params = dict(voxel_size=0.008, mu=0.03, max_w=50, n_buckets=2 ** 12, n_excess=2 ** 10)
    return st


def camera_depth(P, T_wc):
    P = P.astype(np.float64)
    return ((P[..., :3] - T_wc[:3, 3]) @ T_wc[:3, :3])[..., 2]


def compare_raycast(g_ray, o_ray, T_wc, min_cohit=0.995, min_close=0.999):
    """Hit/miss agreement and camera-depth agreement on co-hit pixels.  The
    raycast is a search whose discrete steps depend on binary32 vs binary64
    rounding, so a handful of pixels (silhouettes, grazing rays) may land on a
    different sample; the bar is on the fraction of pixels."""
    P, N = g_ray
    opts, onrm, zc, flags, steps = o_ray
    ghit = P[..., 3] > 0
    ohit = opts[..., 3] > 0
    agree = (ghit == ohit).mean()
    both = ghit & ohit
    z = camera_depth(P, T_wc)
    dz = np.abs(z - zc)[both]
    close = (dz <= DEPTH_TOL).mean() if both.any() else 1.0
    assert agree >= min_cohit, f"hit/miss agreement {agree:.5f}"
    assert close >= min_close, f"co-hit within 0.5 mm {close:.5f}, p99.9 {np.percentile(dz, 99.9):.2e}"
    # normals: valid on the GPU wherever the oracle's are (co-hit pixels), and
    # within 8 degrees of them
    ovalid = both & (onrm[..., 3] > 0)
    if ovalid.any():
        assert (N[..., 3] > 0)[ovalid].mean() >= min_close, "normals missing on the GPU"
    nb = both & (N[..., 3] > 0) & (onrm[..., 3] > 0)
    cosang = (N[..., :3].astype(np.float64) * onrm[..., :3]).sum(-1)[nb]
    if nb.any():
        assert (cosang > 0.99).mean() >= min_close
    return dict(agree=float(agree), close=float(close), median_dz=float(np.median(dz)) if both.any() else 0.0,
                max_dz=float(dz.max()) if both.any() else 0.0)
