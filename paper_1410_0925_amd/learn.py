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
