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


def _block_index(coords, keys):
    """index of each block key (rows of keys) in the sorted block list coords"""
    def k64(c):
        c = np.asarray(c, np.int64) + 32768
        return (c[:, 0] << 32) | (c[:, 1] << 16) | c[:, 2]
    ref = k64(coords)
    q = k64(keys)
    i = np.searchsorted(ref, q)
    assert np.all(i < len(ref)) and np.array_equal(ref[np.minimum(i, len(ref) - 1)], q), \
        "a candidate's block is not allocated"
    return i


def compare_volumes(g_export, o_export, tol=SDF_TOL, cands=None, g_colour=None, o_colour=None):
    """Block sets bit-exact; every voxel's GPU state -- W bit-exact, |dF| <= tol
    and, with colour, the colour bit-exact -- equals the oracle's binary64 state
    or, where one of the voxel's updates had a decision within its binary32
    error bound of a threshold, one of the voxel's other correct states
    (cands = oracle.Scene.export_candidates()).  tol: a number or a function of
    the oracle weight.  Voxels the oracle marks unresolved are counted, not
    compared.  Returns (max |dF| over voxels matching the binary64 state, its
    rms over updated voxels, dict of counts)."""
    gc, gF, gW = g_export
    oc, oF, oW = o_export
    assert gc.shape == oc.shape, (gc.shape, oc.shape)
    assert np.array_equal(gc, oc), "allocated block sets differ"
    tolf = tol if callable(tol) else (lambda w: tol)
    gW64 = gW.astype(np.int64)
    gF64 = gF.astype(np.float64)
    err = np.abs(gF64 - oF)
    ok = (gW64 == oW) & (err <= tolf(oW))
    if g_colour is not None:
        assert g_colour.shape == o_colour.shape, (g_colour.shape, o_colour.shape)
        ok &= np.all(g_colour == o_colour, axis=-1)
    bad = np.argwhere(~ok)
    info = dict(n_alt=0, n_unresolved=0, n_candidate_voxels=0)
    if cands is not None and len(cands["F"]):
        bi = _block_index(gc, cands["key"][:, :3])
        lin = bi.astype(np.int64) * 512 + cands["key"][:, 3]
        info["n_candidate_voxels"] = int(len(np.unique(lin)))
        rows = {}
        for r, x in enumerate(lin.tolist()):
            rows.setdefault(x, []).append(r)
    else:
        rows = {}
    for b, li in bad.tolist():
        rs = rows.get(b * 512 + li)
        what = (f"voxel {li} of block {tuple(gc[b])}: GPU F {gF64[b, li]:.9f} W {gW64[b, li]}, "
                f"oracle F {oF[b, li]:.9f} W {oW[b, li]}")
        assert rs, what + " (the oracle has no other correct state)"
        if any(cands["unresolved"][r] for r in rs):
            info["n_unresolved"] += 1
            continue
        hit = False
        for r in rs:
            w = int(cands["W"][r])
            m = w == gW64[b, li] and abs(gF64[b, li] - cands["F"][r]) <= tolf(np.float64(w))
            if g_colour is not None:
                m = m and bool(np.all(g_colour[b, li] == cands["rgbw"][r]))
            hit = hit or m
        assert hit, what + f"; other states {[(cands['F'][r], int(cands['W'][r])) for r in rs]}"
        info["n_alt"] += 1
    mask = ok & (oW > 0)
    mx = float(err[ok].max()) if ok.any() else 0.0
    rms = float(np.sqrt(np.mean(err[mask] ** 2))) if mask.any() else 0.0
    print(f"volume: {int((oW > 0).sum())} updated voxels, {info['n_candidate_voxels']} with other correct "
          f"states, {info['n_alt']} took another one on the GPU, {info['n_unresolved']} unresolved; "
          f"max |dF| {mx:.2e}", flush=True)
    return mx, rms, info


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


def compare_raycast_exact(g_ray, o_ray, T_wc, tol=DEPTH_TOL):
    """Per-pixel raycast parity on identical volumes.  o_ray: the oracle's
    raycast with alternatives=True.  Every pixel must match one of the ray's
    correct outcomes -- the binary64 march's, or another one reached where a
    sample lay within the binary32 error bound of a rounding boundary (the
    oracle follows both reads): both a miss, or both a hit with camera depths
    within tol (0.5 mm) and, where that outcome has a normal, a GPU normal
    within 8 degrees of it.  Pixels whose march had more branches than the
    oracle follows (flag bit 3) are counted, not compared.  Returns counts and
    the largest |dz| over pixels matched to the binary64 outcome."""
    P, N = g_ray
    opts, onrm, zc, flags, steps, alt = o_ray
    z_g = camera_depth(P, T_wc)
    ghit = P[..., 3] > 0
    gnv = N[..., 3] > 0
    gn = N[..., :3].astype(np.float64)
    # candidates: [H, W, 1 + A]
    c_hit = np.concatenate([(opts[..., 3] > 0)[..., None].astype(np.float64), alt[..., 0]], axis=-1)
    c_z = np.concatenate([zc[..., None], alt[..., 1]], axis=-1)
    c_n = np.concatenate([onrm[..., None, :3], alt[..., 2:5]], axis=-2)
    c_nv = np.concatenate([(onrm[..., 3] > 0)[..., None], alt[..., 5] > 0], axis=-1)
    used = c_hit >= 0
    same = used & ((c_hit > 0) == ghit[..., None])
    dz = np.abs(z_g[..., None] - c_z)
    close = ~ghit[..., None] | (dz <= tol)
    cosang = (gn[..., None, :] * c_n).sum(-1)
    nrm_ok = ~ghit[..., None] | ~c_nv | (gnv[..., None] & (cosang > np.cos(np.radians(8.0))))
    ok_k = same & close & nrm_ok
    unresolved = (flags & 8) > 0
    ok = ok_k.any(-1) | unresolved
    bad = np.argwhere(~ok)
    if len(bad):
        v, u = bad[0]
        dump = __import__("os").environ.get("ITM_DUMP_DIR")
        if dump:   # the failing raycast, for a look on the host
            import glob
            k = len(glob.glob(f"{dump}/raycast_fail_*.npz"))
            b = bad[:64]
            np.savez_compressed(f"{dump}/raycast_fail_{k}.npz", bad=b, T=T_wc, P=P[b[:, 0], b[:, 1]],
                                N=N[b[:, 0], b[:, 1]], opts=opts[b[:, 0], b[:, 1]], onrm=onrm[b[:, 0], b[:, 1]],
                                zc=zc[b[:, 0], b[:, 1]], flags=flags[b[:, 0], b[:, 1]], alt=alt[b[:, 0], b[:, 1]])
        raise AssertionError(
            f"{len(bad)} pixels match none of the oracle's outcomes; first ({u}, {v}): GPU hit {ghit[v, u]} "
            f"z {z_g[v, u]:.6f} n {gn[v, u]} valid {gnv[v, u]}; oracle outcomes "
            f"{[(int(c_hit[v, u, k]), round(float(c_z[v, u, k]), 6)) for k in range(c_hit.shape[-1]) if used[v, u, k]]}")
    prim = ok_k[..., 0] & ghit
    info = dict(pixels=int(ghit.size), hits=int(ghit.sum()),
                branched=int(((flags & 4) > 0).sum()), unresolved=int(unresolved.sum()),
                matched_other=int((~ok_k[..., 0] & ok_k.any(-1)).sum()),
                max_dz_primary=float(dz[..., 0][prim].max()) if prim.any() else 0.0,
                median_dz_primary=float(np.median(dz[..., 0][prim])) if prim.any() else 0.0)
    print("raycast:", info, flush=True)
    return info


def compare_raycast(g_ray, o_ray, T_wc, min_cohit=0.995, min_close=0.999):
    """End-to-end check of a raycast of the GPU's own fused volume against the
    oracle's raycast of its own: hit/miss agreement and camera-depth agreement
    on co-hit pixels as fractions of pixels.  The two volumes may differ where
    a voxel took another correct state (compare_volumes), which moves a few
    marches; per-pixel parity on identical volumes is compare_raycast_exact."""
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
