"""Pins of the refiner oracle (oracle/refine.py): central finite differences of the
FP64 loss, a library conv3d (torch, float64, CPU), torch's bfloat16 rounding and
torch's Adam."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from oracle import refine as R


def _case(seed, nonzero_last=True):
    rng = np.random.default_rng(seed)
    inp = np.stack([rng.uniform(-1, 1, (10, 10, 10)), rng.uniform(0, 1, (10, 10, 10))])
    p = R.init_params(seed)
    W, b = R.unpack(p)
    if nonzero_last:
        W[3, :, 0, :] = rng.standard_normal((27, 16)) * 0.05
        b[:] = rng.standard_normal(b.shape) * 0.01
        b[0, :] = 0.0
    p = R.pack(W, b)
    target = np.clip(inp[0, 1:9, 1:9, 1:9] + rng.normal(0, 0.1, (8, 8, 8)), -1, 1)
    mask = rng.random((8, 8, 8)) < 0.8
    return inp, p, target, mask


def torch_forward(inp, params):
    W, b = R.unpack(params)
    x = torch.zeros((1, 16, 10, 10, 10), dtype=torch.float64)
    x[0, :2] = torch.from_numpy(inp)
    for l in range(4):
        # [tap][co][ci] -> [co][ci][dz][dy][dx]
        w = torch.from_numpy(W[l].reshape(3, 3, 3, 16, 16).transpose(3, 4, 0, 1, 2).copy())
        h = Fn.conv3d(x, w, torch.from_numpy(b[l].copy()))
        if l < 3:
            x = Fn.pad(torch.relu(h), (1, 1, 1, 1, 1, 1))
    out = torch.clamp(torch.from_numpy(inp[0, 1:9, 1:9, 1:9].copy()) + h[0, 0], -1, 1)
    return out.numpy()


def test_forward_matches_library_conv3d():
    inp, p, _, _ = _case(1)
    ours, _ = R.forward(inp, p)
    ref = torch_forward(inp, p)
    assert np.abs(ours - ref).max() < 1e-12


def test_untrained_network_is_identity():
    inp, _, _, _ = _case(2)
    p = R.init_params(7)
    out, _ = R.forward(inp, p)
    assert np.array_equal(out, np.clip(inp[0, 1:9, 1:9, 1:9], -1, 1))


def test_gradient_central_differences():
    inp, p, target, mask = _case(3)
    g, loss = R.backward(inp, p, target, mask)
    rng = np.random.default_rng(4)
    W, b = R.unpack(np.arange(R.N_PARAMS, dtype=np.float64))
    real = []
    for l, ci_n, co_n in ((0, 2, 16), (1, 16, 16), (2, 16, 16), (3, 16, 1)):
        for t in range(27):
            for co in range(co_n):
                for ci in range(ci_n):
                    real.append(int(W[l, t, co, ci]))
    idx = list(rng.choice(real, 60, replace=False)) + [R.N_W + 0, R.N_W + 17, R.N_W + 48]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_fn(R.forward(inp, pp)[0], target, mask) -
              R.loss_fn(R.forward(inp, pm)[0], target, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])
    # padded channels carry no gradient
    gW, gb = R.unpack(g)
    assert np.all(gW[0, :, :, 2:] == 0) and np.all(gW[3, :, 1:, :] == 0) and np.all(gb[3, 1:] == 0)


def test_gradient_matches_autograd():
    inp, p, target, mask = _case(5)
    g, _ = R.backward(inp, p, target, mask)
    W, b = R.unpack(p)
    Wt = [torch.tensor(W[l].reshape(3, 3, 3, 16, 16).transpose(3, 4, 0, 1, 2).copy(), requires_grad=True)
          for l in range(4)]
    bt = [torch.tensor(b[l].copy(), requires_grad=True) for l in range(4)]
    x = torch.zeros((1, 16, 10, 10, 10), dtype=torch.float64)
    x[0, :2] = torch.from_numpy(inp)
    for l in range(4):
        h = Fn.conv3d(x, Wt[l], bt[l])
        if l < 3:
            x = Fn.pad(torch.relu(h), (1, 1, 1, 1, 1, 1))
    out = torch.clamp(torch.from_numpy(inp[0, 1:9, 1:9, 1:9].copy()) + h[0, 0], -1, 1)
    m = torch.from_numpy(mask)
    loss = ((out - torch.from_numpy(target)) ** 2)[m].sum() / m.sum()
    loss.backward()
    gW, gb = R.unpack(g)
    for l in range(4):
        ref = Wt[l].grad.numpy().transpose(2, 3, 4, 0, 1).reshape(27, 16, 16)
        assert np.abs(gW[l] - ref).max() < 1e-12
        assert np.abs(gb[l] - bt[l].grad.numpy()).max() < 1e-12


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(R.bf16(x), ref)


def test_bf16_mode_close_to_exact():
    inp, p, target, mask = _case(8)
    a, _ = R.forward(inp, p)
    b, _ = R.forward(inp, p, bf16_mode=True)
    assert 0 < np.abs(a - b).max() < 5e-2


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(3)]
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, 1):
        opt.zero_grad()
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = R.adam(p, g, m, v, k)
    assert np.abs(p - t.detach().numpy()).max() < 1e-12


def test_forward_batch_is_forward_per_block():
    rng = np.random.default_rng(5)
    p = R.init_params(2)
    W, b = R.unpack(p)
    W[3, :, 0, :] = rng.standard_normal((27, 16)) * 0.05
    b[:3] = rng.standard_normal((3, 16)) * 0.05
    p = R.pack(W, b)
    inp = np.stack([np.clip(rng.normal(0.2, 0.6, (3, 10, 10, 10)), -1, 1), rng.random((3, 10, 10, 10))], axis=1)
    for mode in (False, True):
        got = R.forward_batch(inp, p, bf16_mode=mode)
        want = np.stack([R.forward(inp[i], p, bf16_mode=mode)[0] for i in range(3)])
        assert np.abs(got - want).max() < 1e-12
