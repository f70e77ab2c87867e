"""Learned block refiner: training pairs produced by the fusion path itself and a
training loop on the library's MFMA kernels (through the C ABI only).

A pair is a block allocated after the first `n_early` frames of a stream: the
input is its network input at that time (F and W / max_w with a one-voxel halo),
the target is its F after `n_late` frames, supervised where the late weight is
positive.
"""
from __future__ import annotations

import numpy as np

from . import Refiner, Scene


def make_pairs(stream, n_early=5, n_late=100, fmt="f32"):
    """Returns (inputs [n, 2000], target [n, 512], mask [n, 512] uint8, coords),
    the first three as torch tensors on the GPU."""
    import torch
    K = tuple(stream.intrinsics) + (stream.width, stream.height)
    depth = torch.from_numpy(np.ascontiguousarray(stream.depth[:n_late])).cuda()
    with Scene.from_params(stream.params, fmt=fmt) as sc:
        for f in range(n_early):
            sc.integrate(depth[f], K, stream.T_wc[f])
        coords, _, _ = sc.export(values=False)
        inputs = sc.gather(coords)
        for f in range(n_early, n_late):
            sc.integrate(depth[f], K, stream.T_wc[f])
        c2, F2, W2 = sc.export()
    key = lambda c: (c[:, 0].astype(np.int64) << 40) + (c[:, 1].astype(np.int64) << 20) + c[:, 2]
    k2 = key(c2.astype(np.int64) + 2 ** 19)
    idx = np.searchsorted(k2, key(coords.astype(np.int64) + 2 ** 19))
    assert np.array_equal(c2[idx], coords), "blocks are never removed"
    target = torch.from_numpy(np.ascontiguousarray(F2[idx])).cuda()
    mask = torch.from_numpy((W2[idx] > 0).astype(np.uint8)).cuda()
    return inputs, target, mask, coords


def concat_pairs(pairs):
    import torch
    return tuple(torch.cat([p[i] for p in pairs]) for i in range(3))


def train(refiner: Refiner, inputs, target, mask, steps, batch=256, lr=1e-3, seed=0, log_every=0):
    """Adam on random mini-batches; returns the loss of every step (float32)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = inputs.shape[0]
    losses = torch.empty(steps, dtype=torch.float32, device="cuda")
    for s in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).cuda()
        refiner.train_step(inputs[idx].contiguous(), target[idx].contiguous(), mask[idx].contiguous(), lr,
                           loss=losses[s:s + 1])
        if log_every and (s + 1) % log_every == 0:
            print(f"step {s + 1}: loss {float(losses[s]):.3e}", flush=True)
    return losses.cpu().numpy()


def evaluate(refiner: Refiner, inputs, target, mask, batch=1024):
    """RMS error against the target over supervised voxels, without and with the
    network: (rms_plain, rms_refined)."""
    import torch
    outs = [refiner.forward(inputs[i:i + batch].contiguous()) for i in range(0, inputs.shape[0], batch)]
    out = torch.cat(outs)
    centre = inputs.view(-1, 2, 10, 10, 10)[:, 0, 1:9, 1:9, 1:9].reshape(-1, 512)
    m = mask.bool()
    rms_plain = torch.sqrt(torch.mean((centre - target)[m] ** 2)).item()
    rms_ref = torch.sqrt(torch.mean((out - target)[m] ** 2)).item()
    return rms_plain, rms_ref


def held_out_errors(refiner: Refiner, inputs, target, w_late, F_truth, w_gate=0.1, batch=1024):
    """Errors over the band voxels (|F_late| < 1, W_late > 0) of the gated blocks
    (largest early weight / max_w below w_gate): RMS of F_early against F_late,
    of the network's output against F_late, and both against F_truth (the
    analytic signed distance / mu, clamped to [-1, 1])."""
    import torch
    outs = [refiner.forward(inputs[i:i + batch].contiguous()) for i in range(0, inputs.shape[0], batch)]
    out = torch.cat(outs)
    x = inputs.view(-1, 2, 10, 10, 10)
    centre = x[:, 0, 1:9, 1:9, 1:9].reshape(-1, 512)
    w_early_max = x[:, 1, 1:9, 1:9, 1:9].reshape(-1, 512).amax(dim=1)
    gated = (w_early_max < w_gate)[:, None]
    band = (target.abs() < 1) & (w_late > 0) & gated
    rms = lambda a, b: torch.sqrt(torch.mean((a - b)[band] ** 2)).item()
    return {"voxels": int(band.sum().item()), "gated_blocks": int(gated.sum().item()),
            "rms_plain_vs_late": rms(centre, target), "rms_refined_vs_late": rms(out, target),
            "rms_plain_vs_analytic": rms(centre, F_truth), "rms_refined_vs_analytic": rms(out, F_truth)}


def analytic_F(stream, coords, mu):
    """the scene's signed distance at every voxel of the blocks (world v * s), / mu,
    clamped to [-1, 1], as [n, 512] (voxel order lx + 8 ly + 64 lz)"""
    s = float(np.float32(stream.params["voxel_size"]))
    l = np.arange(512)
    off = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1)
    out = np.empty((len(coords), 512), np.float32)
    for i in range(0, len(coords), 4096):
        c = coords[i:i + 4096].astype(np.int64)
        v = (8 * c[:, None, :] + off[None]) * s
        out[i:i + 4096] = np.clip(stream.scene.signed_distance(v) / mu, -1, 1)
    return out


def init_params(seed: int) -> np.ndarray:
    """Initial parameter vector (the library's layout): He-normal weights for
    layers 1-3 over their real fan-in (27 taps x 2 or 16 channels), layer 4 and
    the biases zero, so the untrained network returns its input F."""
    rng = np.random.default_rng(seed)
    W = np.zeros((4, 27, 16, 16))
    W[0, :, :, :2] = rng.standard_normal((27, 16, 2)) * np.sqrt(2.0 / (27 * 2))
    W[1] = rng.standard_normal((27, 16, 16)) * np.sqrt(2.0 / (27 * 16))
    W[2] = rng.standard_normal((27, 16, 16)) * np.sqrt(2.0 / (27 * 16))
    return np.concatenate([W.ravel(), np.zeros(4 * 16)]).astype(np.float32)


def c4_recipe(n_rooms=50, n_train=40, n_frames=100, n_early=5, steps=20000, batch=256, lr=1e-3, seed=0,
              w_threshold=10.0, log=print):
    """Rooms 1000 .. 1000 + n_rooms - 1 (vga-style, n_frames each): pairs of every
    block allocated after n_early frames (input: its haloed early TSDF; target:
    its F after n_frames); train on the first n_train rooms, evaluate on the
    rest.  Returns a dict of the run's numbers."""
    import time
    import torch
    from synth import make_stream
    t0 = time.perf_counter()
    train_sets, held = [], []
    for r in range(n_rooms):
        st = make_stream("room", n_frames=n_frames, seed=1000 + r, cache=False)
        inputs, target, mask, coords = make_pairs(st, n_early, n_frames)
        max_w = st.params["max_w"]
        if r < n_train:
            train_sets.append((inputs, target, mask))
        else:
            mu = st.params["mu"]
            truth = torch.from_numpy(analytic_F(st, coords, mu)).cuda()
            held.append((inputs, target, mask, truth))
        log(f"room {1000 + r}: {inputs.shape[0]} blocks ({time.perf_counter() - t0:.0f} s)")
        del st
    inputs, target, mask = concat_pairs(train_sets)
    del train_sets
    n_train_blocks = int(inputs.shape[0])
    ref = Refiner(init_params(seed))
    t1 = time.perf_counter()
    losses = train(ref, inputs, target, mask, steps, batch=batch, lr=lr, seed=seed,
                   log_every=max(1, steps // 10))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del inputs, target, mask
    hi = torch.cat([h[0] for h in held])
    ht = torch.cat([h[1] for h in held])
    hm = torch.cat([h[2] for h in held])
    htr = torch.cat([h[3] for h in held])
    # W_late > 0 where the mask is set
    errs = held_out_errors(ref, hi, ht, hm, htr, w_gate=w_threshold / max_w)
    out = {"rooms": n_rooms, "train_rooms": n_train, "frames": n_frames, "early_frames": n_early,
           "train_blocks": n_train_blocks, "held_out_blocks": int(hi.shape[0]), "steps": steps, "batch": batch,
           "lr": lr, "train_s": t_train, "loss_first_100": float(np.mean(losses[:100])),
           "loss_last_100": float(np.mean(losses[-100:])), "params": ref.params().tolist(), **errs}
    ref.close()
    return out


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="the learned refiner's training recipe on generated rooms")
    ap.add_argument("--rooms", type=int, default=50)
    ap.add_argument("--train-rooms", type=int, default=40)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--early", type=int, default=5)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None, help="write the numbers (and the trained parameters) as JSON here")
    a = ap.parse_args()
    res = c4_recipe(a.rooms, a.train_rooms, a.frames, a.early, a.steps, a.batch, a.lr,
                    log=lambda m: print(m, flush=True))
    summary = {k: v for k, v in res.items() if k != "params"}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    _main()
