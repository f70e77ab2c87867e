"""Learned refiner on the GPU (bf16 MFMA kernels through the C ABI) against the
FP64 oracle in bf16 mode (identical bf16-rounded operands), plus training and the
held-out gain of the trained network over the plain few-frame fusion."""
import numpy as np
import pytest

from oracle import refine as R
from synth import make_stream
from tests.gpu_util import fuse_gpu, fuse_oracle, gpu

pytestmark = pytest.mark.gpu


def _params(seed):
    rng = np.random.default_rng(seed)
    p = R.init_params(seed)
    W, b = R.unpack(p)
    W[3, :, 0, :] = rng.standard_normal((27, 16)) * 0.05
    b[:3] = rng.standard_normal((3, 16)) * 0.05
    b[3, 0] = 0.01
    return R.pack(W, b).astype(np.float32)


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    F = np.clip(rng.normal(0.3, 0.6, (n, 10, 10, 10)), -1, 1)
    W = rng.integers(0, 6, (n, 10, 10, 10)) / 100.0
    inp = np.stack([F, W], axis=1).astype(np.float32)
    target = np.clip(F[:, 1:9, 1:9, 1:9] + rng.normal(0, 0.2, (n, 8, 8, 8)), -1, 1).astype(np.float32)
    mask = (rng.random((n, 8, 8, 8)) < 0.7).astype(np.uint8)
    return inp, target, mask


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_parity():
    itm, torch = gpu()
    p = _params(1)
    inp, _, _ = _inputs(2, 6)
    ref = itm.Refiner(p)
    out = ref.forward(torch.from_numpy(inp.reshape(6, 2000)).cuda()).cpu().numpy()
    want = np.stack([R.forward(inp[i].astype(np.float64), p.astype(np.float64), bf16_mode=True)[0]
                     for i in range(6)]).reshape(6, 512)
    err = rel_l2(out - inp[:, 0, 1:9, 1:9, 1:9].reshape(6, 512), want - inp[:, 0, 1:9, 1:9, 1:9].reshape(6, 512))
    print(f"forward residual rel L2 {err:.2e}, max |dF| {np.abs(out - want).max():.2e}")
    assert err < 1e-3
    assert np.abs(out - want).max() < 1e-3


def test_gradient_parity():
    itm, torch = gpu()
    p = _params(3)
    inp, target, mask = _inputs(4, 4)
    ref = itm.Refiner(p)
    g, loss = ref.gradient(torch.from_numpy(inp.reshape(4, 2000)).cuda(),
                           torch.from_numpy(target.reshape(4, 512)).cuda(),
                           torch.from_numpy(mask.reshape(4, 512)).cuda())
    g = g.cpu().numpy().astype(np.float64)
    want, wloss = R.batch_grad([x.astype(np.float64) for x in inp], p.astype(np.float64), target.astype(np.float64),
                               mask.astype(bool), bf16_mode=True)
    assert abs(float(loss.cpu()) - wloss) <= 1e-4 * wloss
    gW, gb = R.unpack(g)
    wW, wb = R.unpack(want)
    for l in range(4):
        e = rel_l2(gW[l], wW[l])
        eb = rel_l2(gb[l], wb[l])
        print(f"layer {l + 1}: dW rel L2 {e:.2e}, db rel L2 {eb:.2e}")
        assert e < 1e-3 and eb < 1e-3
    # channels outside a layer's width stay exactly zero
    assert np.all(gW[0, :, :, 2:] == 0) and np.all(gW[3, :, 1:, :] == 0) and np.all(gb[3, 1:] == 0)


def test_adam_step_parity():
    itm, torch = gpu()
    p = _params(5)
    inp, target, mask = _inputs(6, 3)
    ref = itm.Refiner(p)
    args = [torch.from_numpy(x.reshape(3, -1)).cuda() for x in (inp, target, mask)]
    g, _ = ref.gradient(*args)
    g = g.cpu().numpy().astype(np.float64)
    ref.train_step(*args, 1e-3)
    got = ref.params().astype(np.float64)
    want, _, _ = R.adam(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    assert np.abs(got - want).max() < 1e-6


def test_gather_parity():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=4)
    o, _, _ = fuse_oracle(st)
    oc, oF, oW = o.export()
    # the oracle's volume loaded into the GPU scene (binary32 values): both
    # sides hold the same voxels
    oF = oF.astype(np.float32).astype(np.float64)
    g = itm.Scene.from_params(st.params)
    g.import_blocks(oc, oF.astype(np.float32), oW.astype(np.float32))
    pick = oc[:: max(1, len(oc) // 40)]
    got = g.gather(pick).cpu().numpy().reshape(-1, 2, 10, 10, 10)
    vol = {tuple(c): (f.reshape(8, 8, 8), w.reshape(8, 8, 8)) for c, f, w in zip(oc.tolist(), oF, oW)}
    max_w = st.params["max_w"]
    for b, (kx, ky, kz) in enumerate(pick.tolist()):
        want = np.zeros((2, 10, 10, 10))
        for z in range(10):
            for y in range(10):
                for x in range(10):
                    v = (8 * kx - 1 + x, 8 * ky - 1 + y, 8 * kz - 1 + z)
                    blk = tuple(c // 8 for c in v)
                    if blk in vol:
                        f, w = vol[blk]
                        want[0, z, y, x] = f[v[2] % 8, v[1] % 8, v[0] % 8]
                        want[1, z, y, x] = w[v[2] % 8, v[1] % 8, v[0] % 8] / max_w
                    else:
                        want[0, z, y, x] = 1.0
        assert np.abs(got[b, 0] - want[0]).max() <= 1e-5
        assert np.abs(got[b, 1] - want[1]).max() <= 1e-6


def test_training_gain_on_held_out_room():
    """Trained on pairs from 3 rooms (5 frames -> 60 frames), the network moves the
    5-frame TSDF of a held-out room closer to its 60-frame TSDF."""
    itm, torch = gpu()
    from paper_1410_0925_amd import learn
    train_pairs = [learn.make_pairs(make_stream("room", n_frames=60, seed=s), 5, 60) for s in (1000, 1001, 1002)]
    held = learn.make_pairs(make_stream("room", n_frames=60, seed=1040), 5, 60)
    inputs, target, mask = learn.concat_pairs(train_pairs)
    print(f"training blocks {inputs.shape[0]}, held-out blocks {held[0].shape[0]}", flush=True)
    ref = itm.Refiner(R.init_params(0).astype(np.float32))
    before = learn.evaluate(ref, *held[:3])
    losses = learn.train(ref, inputs, target, mask, steps=600, batch=128, lr=1e-3)
    after = learn.evaluate(ref, *held[:3])
    print(f"loss first 20 {losses[:20].mean():.4e} last 20 {losses[-20:].mean():.4e}; held-out RMS "
          f"plain {after[0]:.4e} refined {after[1]:.4e} (untrained {before[1]:.4e})")
    assert abs(before[0] - before[1]) < 1e-6          # untrained network is the identity
    assert losses[-20:].mean() < 0.9 * losses[:20].mean()
    assert after[1] < after[0]


def test_gated_inference_in_integrate():
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=3)
    p = _params(7)
    ref = itm.Refiner(p)
    sc = itm.Scene.from_params(st.params)
    sc.set_refiner(ref, w_threshold=3.0)
    K = tuple(st.intrinsics) + (st.width, st.height)
    for f in range(3):
        sc.integrate(torch.from_numpy(st.depth[f]).cuda(), K, st.T_wc[f])
    coords, Fr, flags = sc.export_refined()
    c2, F, W = sc.export()
    assert np.array_equal(coords, c2)
    vis = sc.stats()["n_visible_last"]
    assert 0 < flags.sum() <= vis
    assert np.all(W[flags].max(axis=1) < 3.0)
    # refined values equal the network applied to the gathered blocks (half storage)
    sel = coords[flags][:20]
    out = ref.forward(sc.gather(sel)).cpu().numpy()
    assert np.abs(out - Fr[flags][:20]).max() <= 1e-3
    # unrefined blocks export the plain F
    assert np.array_equal(Fr[~flags], F[~flags])


def haloed_inputs(coords, F, Wt, idx, max_w):
    """network inputs [len(idx), 2, 10, 10, 10] of blocks idx of a volume (coords
    [n, 3], F / W [n, 512]): F and W / max_w on voxels 8k-1 .. 8k+8, voxels of
    absent blocks reading (1, 0)"""
    pos = {tuple(c): i for i, c in enumerate(coords.tolist())}
    F8 = F.reshape(-1, 8, 8, 8)          # [z][y][x]
    W8 = Wt.reshape(-1, 8, 8, 8).astype(np.float64) / max_w
    out = np.zeros((len(idx), 2, 10, 10, 10))
    out[:, 0] = 1.0
    for n, b in enumerate(idx):
        kx, ky, kz = coords[b]
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    j = pos.get((kx + dx, ky + dy, kz + dz))
                    if j is None:
                        continue
                    # the part of neighbour j inside the 10^3 window
                    sl_dst, sl_src = [], []
                    for d in (dz, dy, dx):
                        if d == -1:
                            sl_dst.append(slice(0, 1)); sl_src.append(slice(7, 8))
                        elif d == 0:
                            sl_dst.append(slice(1, 9)); sl_src.append(slice(0, 8))
                        else:
                            sl_dst.append(slice(9, 10)); sl_src.append(slice(0, 1))
                    out[n, 0][tuple(sl_dst)] = F8[j][tuple(sl_src)]
                    out[n, 1][tuple(sl_dst)] = W8[j][tuple(sl_src)]
    return out


def test_raycast_reads_refined_blocks():
    """The raycast prefers a refined block's F: a volume the oracle fused from 2
    frames (every block below the weight gate) is loaded into the GPU scene, the
    refiner runs over it (itm_refine_visible), and the GPU raycast is held to the
    oracle's raycast of the same volume with the gated blocks replaced by the
    oracle's bf16-mode forward pass (stored as binary16, as the side buffer
    is).  The network's values differ between the two by bf16 accumulation
    order, so the bar is on the fraction of pixels within 0.5 mm; the refined
    raycast must also differ from the plain one."""
    import oracle
    from tests.gpu_util import K_of, camera_depth
    itm, torch = gpu()
    st = make_stream("tiny", n_frames=2)
    o, _, _ = fuse_oracle(st)
    oc, oF, oW = o.export()
    F32 = oF.astype(np.float32)
    g = itm.Scene.from_params(st.params)
    g.import_blocks(oc, F32, oW.astype(np.float32))
    K = K_of(st)
    T = st.T_wc[1]
    p0, _ = g.raycast(K, T)
    p = _params(7)
    ref = itm.Refiner(p)
    thr = 10.0
    g.set_refiner(ref, thr)
    g.refine_visible()
    p1, n1 = g.raycast(K, T)
    torch.cuda.synchronize()
    gated = np.flatnonzero(oW.max(axis=1) < thr)
    assert len(gated) == len(oc)          # two frames: every block is below the gate
    inp = haloed_inputs(oc, F32.astype(np.float64), oW, gated, st.params["max_w"])
    Fref = F32.astype(np.float64).copy()
    for k in range(0, len(gated), 256):
        Fref[gated[k:k + 256]] = R.forward_batch(inp[k:k + 256], p.astype(np.float64),
                                                 bf16_mode=True).reshape(-1, 512)
    Fref = Fref.astype(np.float16).astype(np.float64)
    # the GPU's refined blocks (the side buffer) against the oracle's forward
    gc, gF, flags = g.export_refined()
    assert flags.all() and np.array_equal(gc, oc)
    print(f"refined F: max |dF| {np.abs(gF - Fref).max():.2e}, moved by the net {np.abs(Fref - F32).max():.2e}")
    assert np.abs(gF - Fref).max() < 5e-3   # bf16 sums in another order, then binary16
    o2 = oracle.Scene.from_params(st.params)
    o2.import_blocks(oc, Fref, oW)
    opts, onrm, zc, fl, _ = o2.raycast(st.width, st.height, st.intrinsics, T)
    P1 = p1.cpu().numpy()
    ghit, ohit = P1[..., 3] > 0, opts[..., 3] > 0
    z1 = camera_depth(P1, T)
    both = ghit & ohit
    close = (np.abs(z1 - zc)[both] <= 5e-4).mean()
    print(f"refined raycast: hit/miss agree {(ghit == ohit).mean():.5f}, co-hit within 0.5 mm {close:.5f}")
    assert (ghit == ohit).mean() >= 0.995 and close >= 0.995
    # and the refiner changed what the raycast sees
    P0 = p0.cpu().numpy()
    z0 = camera_depth(P0, T)
    moved = (np.abs(z1 - z0) > 1e-4)[both & (P0[..., 3] > 0)].mean()
    print(f"pixels moved by more than 0.1 mm by the refiner: {moved:.3f}")
    assert moved > 0.05
    # detached: the plain raycast again, bit for bit
    g.set_refiner(None)
    p2, _ = g.raycast(K, T)
    assert torch.equal(p2, p0)
    g.close()
    ref.close()
