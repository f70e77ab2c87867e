"""FP64 oracle of the learned block refiner (test infrastructure only).

The refiner is not in the paper: it is a small 3D convolutional network that maps
a block's few-frame TSDF (with a one-voxel halo) to an estimate of the TSDF the
plain running average of the paper's section "Integration" reaches after many
frames.  Architecture (every layer a 3^3 convolution from a 10^3 grid to the 8^3
block, i.e. valid on the haloed input and zero-padded afterwards):

    in  [2, 10^3]: F, W / max_w            (neighbour voxels of absent blocks: F=1, W=0)
    L1  2 -> 16, ReLU
    L2 16 -> 16, ReLU
    L3 16 -> 16, ReLU
    L4 16 ->  1
    F_out = clamp(F_centre + L4, -1, 1)
    loss  = sum over voxels with target weight > 0 of (F_out - F_target)^2 / count

Parameter vector (float32 on the wire), the layout the library uses:
    for layer l in 1..4: W_l[tap][co][ci], tap = dz*9 + dy*3 + dx, co, ci in 0..15
    then b_l[co] for l in 1..4
Channels beyond a layer's real width (L1 inputs 2..15, L4 outputs 1..15) hold 0.

`bf16=True` rounds, as the MFMA kernels do, every matrix operand to bfloat16 (the
network input, weights, hidden activations after ReLU, and the back-propagated
gradients before they enter a product); sums are exact (binary64) here.
"""
from __future__ import annotations

import numpy as np

C = 16
TAPS = 27
N_LAYERS = 4
N_W = N_LAYERS * TAPS * C * C
N_PARAMS = N_W + N_LAYERS * C


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def unpack(params):
    p = np.asarray(params, np.float64)
    W = p[:N_W].reshape(N_LAYERS, TAPS, C, C)          # [l][tap][co][ci]
    b = p[N_W:].reshape(N_LAYERS, C)
    return W, b


def pack(W, b):
    return np.concatenate([np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64).ravel()])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights for L1..L3 on their real fan-in, L4 and biases zero (the
    untrained network is the identity F_out = F_centre)."""
    rng = np.random.default_rng(seed)
    W = np.zeros((N_LAYERS, TAPS, C, C))
    b = np.zeros((N_LAYERS, C))
    W[0, :, :, :2] = rng.standard_normal((TAPS, C, 2)) * np.sqrt(2.0 / (TAPS * 2))
    for l in (1, 2):
        W[l] = rng.standard_normal((TAPS, C, C)) * np.sqrt(2.0 / (TAPS * C))
    return pack(W, b).astype(np.float32).astype(np.float64)


def _taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield dz * 9 + dy * 3 + dx, dz, dy, dx


def conv(x10, Wl, bl):
    """out[co, v] = b[co] + sum_tap sum_ci x10[ci, v + tap] W[tap, co, ci]
    for v in the 8^3 block (x10 is the 10^3 grid)."""
    out = np.zeros((C, 8, 8, 8)) + bl[:, None, None, None]
    for t, dz, dy, dx in _taps():
        xs = x10[:, dz:dz + 8, dy:dy + 8, dx:dx + 8]            # [ci, 8,8,8]
        out += np.einsum("oi,izyx->ozyx", Wl[t], xs)
    return out


def pad(a8):
    x = np.zeros((a8.shape[0], 10, 10, 10))
    x[:, 1:9, 1:9, 1:9] = a8
    return x


def forward(inp, params, bf16_mode=False):
    """inp: [2, 10, 10, 10] (F, W/max_w).  Returns (F_out [8,8,8], cache)."""
    rnd = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    W, b = unpack(params)
    W = rnd(W)
    x0 = np.zeros((C, 10, 10, 10))
    x0[:2] = rnd(inp)
    xs, pre = [x0], []
    for l in range(N_LAYERS):
        h = conv(xs[-1], W[l], b[l])
        pre.append(h)
        if l < N_LAYERS - 1:
            xs.append(pad(rnd(np.maximum(h, 0.0))))
    delta = pre[-1][0]
    centre = np.asarray(inp[0], np.float64)[1:9, 1:9, 1:9]
    z = centre + delta
    F_out = np.clip(z, -1.0, 1.0)
    return F_out, dict(xs=xs, pre=pre, W=W, z=z)


def forward_batch(inp, params, bf16_mode=False):
    """forward() over a batch: inp [n, 2, 10, 10, 10] -> F_out [n, 8, 8, 8]
    (the same sums, the block index carried along)"""
    rnd = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    W, b = unpack(params)
    W = rnd(W)
    inp = np.asarray(inp, np.float64)
    n = inp.shape[0]
    x = np.zeros((n, C, 10, 10, 10))
    x[:, :2] = rnd(inp)
    for l in range(N_LAYERS):
        h = np.zeros((n, C, 8, 8, 8)) + b[l][None, :, None, None, None]
        for t, dz, dy, dx in _taps():
            xs = np.ascontiguousarray(x[:, :, dz:dz + 8, dy:dy + 8, dx:dx + 8]).reshape(n, C, 512)
            h += np.matmul(W[l][t], xs).reshape(n, C, 8, 8, 8)
        if l < N_LAYERS - 1:
            x = np.zeros((n, C, 10, 10, 10))
            x[:, :, 1:9, 1:9, 1:9] = rnd(np.maximum(h, 0.0))
    return np.clip(inp[:, 0, 1:9, 1:9, 1:9] + h[:, 0], -1.0, 1.0)


def loss_fn(F_out, target, mask):
    m = np.asarray(mask, bool)
    n = max(int(m.sum()), 1)
    return float(np.sum(((F_out - target) ** 2)[m]) / n)


def backward(inp, params, target, mask, bf16_mode=False, n_norm=None):
    """Gradient of loss_fn w.r.t. the parameter vector (same layout).  n_norm
    overrides the loss normaliser (a batch divides by its total count)."""
    rnd = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    F_out, cache = forward(inp, params, bf16_mode)
    W, xs, pre, z = cache["W"], cache["xs"], cache["pre"], cache["z"]
    m = np.asarray(mask, bool)
    n = n_norm if n_norm is not None else max(int(m.sum()), 1)
    g = np.where(m, 2.0 * (F_out - target) / n, 0.0)
    g = np.where((z > -1.0) & (z < 1.0), g, 0.0)               # clamp passes inside only
    d = np.zeros((C, 8, 8, 8))
    d[0] = g
    dW = np.zeros_like(W)
    db = np.zeros((N_LAYERS, C))
    for l in range(N_LAYERS - 1, -1, -1):
        dq = rnd(d)
        db[l] = dq.sum(axis=(1, 2, 3))
        x = xs[l]
        for t, dz, dy, dx in _taps():
            dW[l, t] = np.einsum("ozyx,izyx->oi", dq, x[:, dz:dz + 8, dy:dy + 8, dx:dx + 8])
        if l == 0:
            break
        # gradient w.r.t. the 10^3 input grid, then its 8^3 interior
        dx10 = np.zeros((C, 10, 10, 10))
        for t, dz, dy, dx_ in _taps():
            dx10[:, dz:dz + 8, dy:dy + 8, dx_:dx_ + 8] += np.einsum("oi,ozyx->izyx", W[l, t], dq)
        da = dx10[:, 1:9, 1:9, 1:9]
        d = np.where(pre[l - 1] > 0.0, da, 0.0)
    return pack(dW, db), loss_fn(F_out, target, m)


def batch_grad(inputs, params, targets, masks, bf16_mode=False):
    """Mean-over-valid-voxels loss of a batch of blocks and its gradient.  Each
    block back-propagates the unnormalised 2 (F_out - F_target) (so that, in
    bf16 mode, gradients are rounded where the kernels round them) and the sum
    is divided by the batch's count of supervised voxels at the end."""
    n = max(int(sum(np.asarray(mk, bool).sum() for mk in masks)), 1)
    grad = np.zeros(N_PARAMS)
    loss = 0.0
    for inp, t, mk in zip(inputs, targets, masks):
        g, _ = backward(inp, params, t, mk, bf16_mode, n_norm=1.0)
        grad += g
        F_out, _ = forward(inp, params, bf16_mode)
        loss += float(np.sum(((F_out - t) ** 2)[np.asarray(mk, bool)]))
    return grad / n, loss / n


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
