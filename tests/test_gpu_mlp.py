"""Warm-start network kernels (BF16 MFMA, FP32 sums) against the FP64
reference network: forward outputs, loss and every parameter gradient, Adam
updates, and training on a smooth target.  Two references: one that rounds
what the kernels hold in bfloat16 (tight bound: the kernels differ from it
only by FP32 instead of FP64 sums and rare bf16 rounding flips) and the plain
FP64 network (loose bound from bfloat16 resolution, 2^-8 relative per
rounding, accumulated over five layers)."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _data(B, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.stack([rng.uniform(0.1, 1.0, B), rng.uniform(-1, 1, B), rng.uniform(0, 1, B)], 1)
    t = np.stack([np.sin(3 * x[:, 2] + k) * x[:, 0] + 0.3 * x[:, 1] * k for k in range(6)], 1)
    return x.astype(np.float32), t.astype(np.float32)


def _net(B, p):
    from paper_0705_0497_amd.binding import Network
    return Network(B, params=p.astype(np.float32))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B", [1, 200, 3001])
def test_forward_matches_reference(B):
    import torch
    p = M.init_params(7).astype(np.float32).astype(np.float64)
    x, _ = _data(B)
    print(f"mlp forward B={B}", flush=True)
    net = _net(max(B, 64), p)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    y16, _ = M.forward(p, x.astype(np.float64), emulate=True)
    y64, _ = M.forward(p, x.astype(np.float64))
    assert _rel(y, y16) < 2e-3
    assert np.max(np.abs(y - y16)) < 5e-3 * max(1.0, np.max(np.abs(y16)))
    assert _rel(y, y64) < 3e-2


@pytest.mark.parametrize("B", [37, 333, 5000])
def test_loss_and_gradients_match_reference(B):
    import torch
    p = M.init_params(9).astype(np.float32).astype(np.float64)
    x, t = _data(B, seed=B)
    print(f"mlp backward B={B}", flush=True)
    net = _net(B, p)
    loss = net.backward(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads().astype(np.float64)
    l16, g16 = M.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64), emulate=True)
    l64, g64 = M.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - l16) <= 1e-4 * l16
    assert abs(loss - l64) <= 2e-2 * l64
    k = 0
    for l, (o, i) in enumerate(M.SIZES):
        for name, n in (("W", o * i), ("b", o)):
            a, r16, r64 = g[k:k + n], g16[k:k + n], g64[k:k + n]
            assert _rel(a, r16) < 5e-3, (l, name, _rel(a, r16))
            assert _rel(a, r64) < 6e-2, (l, name, _rel(a, r64))
            k += n
    assert k == M.NPARAM


def test_adam_steps_follow_reference():
    import torch
    p0 = M.init_params(4).astype(np.float32).astype(np.float64)
    x, t = _data(256, seed=3)
    net = _net(256, p0)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    lr = 1e-3
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k in range(1, 4):
        net.backward(xd, td, want_loss=False)
        net.adam(lr)
        _, g = M.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64), emulate=True)
        p, m, v = M.adam(p, g, m, v, k, lr)
    q = net.params().astype(np.float64)
    d = np.abs(q - p)
    assert np.max(np.abs(q - p0)) > 2 * lr                       # the weights did move
    assert np.mean(d < 0.05 * lr) > 0.99                          # the same steps almost everywhere
    assert np.max(d) <= 6 * lr


def test_training_reduces_the_loss():
    import torch
    p = M.init_params(5).astype(np.float32)
    x, t = _data(4096, seed=8)
    net = _net(4096, p)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    first = net.backward(xd, td)
    for _ in range(300):
        net.backward(xd, td, want_loss=False)
        net.adam(2e-3)
    last = net.backward(xd, td)
    print(f"mlp training loss {first:.4g} -> {last:.4g}", flush=True)
    assert last < 0.05 * first
    y = net.forward(xd).cpu().numpy()
    assert abs(float(np.mean((y - t) ** 2)) - last) < 0.05 * last
