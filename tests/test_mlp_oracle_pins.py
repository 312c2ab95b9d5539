"""Pins of the FP64 warm-start network reference (oracle/mlp.py) against what
mathematics fixes: central finite differences of the loss, closed forms of
GELU and of Adam's first steps, bfloat16 rounding as torch implements it."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _problem(seed=3, B=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = M.init_params(seed)
    x = rng.uniform(-1, 1, size=(B, 3))
    t = rng.normal(size=(B, 6))
    return p, x, t


def test_parameter_count():
    assert M.NPARAM == 3 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 6 + 6 == 199942


def test_gradient_matches_central_differences():
    p, x, t = _problem()
    _, g = M.loss_and_grad(p, x, t)
    rng = np.random.Generator(np.random.PCG64(11))
    # a sample in every tensor: first layer, hidden layers, output layer, biases
    offs, k = [], 0
    for o, i in M.SIZES:
        offs += list(k + rng.integers(0, o * i, 6)) + list(k + o * i + rng.integers(0, o, 2))
        k += o * i + o
    h = 1e-5
    for j in offs:
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (M.loss_and_grad(pp, x, t)[0] - M.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 + 1e-5 * abs(fd), (j, fd, g[j])


def test_gelu_closed_forms():
    from scipy.stats import norm
    z = np.linspace(-6, 6, 97)
    np.testing.assert_allclose(M.gelu(z), z * norm.cdf(z), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(M.gelu_prime(z), norm.cdf(z) + z * norm.pdf(z), rtol=1e-13, atol=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0 and M.gelu_prime(np.array([0.0]))[0] == 0.5
    # derivative against a central difference of the function itself
    h = 1e-6
    np.testing.assert_allclose((M.gelu(z + h) - M.gelu(z - h)) / (2 * h), M.gelu_prime(z), atol=1e-8)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.Generator(np.random.PCG64(5))
    v = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(v), ref)
    assert M.bf16(np.float32(1.0 + 2 ** -8)) == 1.0                 # tie to even
    assert M.bf16(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6   # tie to even, upwards


def test_adam_first_steps_closed_form():
    rng = np.random.Generator(np.random.PCG64(2))
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = M.adam(p0, g, np.zeros(50), np.zeros(50), 1, lr)
    np.testing.assert_allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected step unchanged
    p2, _, _ = M.adam(p1, g, m, v, 2, lr)
    np.testing.assert_allclose(p2 - p1, p1 - p0, rtol=1e-9, atol=1e-15)


def test_zero_weights_output_the_last_bias_and_emulation_is_close():
    p, x, t = _problem()
    q = p.copy()
    W4 = M.unflatten(q)[4][0]
    W4[:] = 0.0
    y, _ = M.forward(q, x)
    np.testing.assert_array_equal(y, np.broadcast_to(M.unflatten(q)[4][1], y.shape))
    # bfloat16 emulation stays within a few bf16 steps of the exact network
    y64, _ = M.forward(p, x)
    y16, _ = M.forward(p, x, emulate=True)
    assert np.max(np.abs(y16 - y64)) < 0.05 * np.max(np.abs(y64))
    _, g64 = M.loss_and_grad(p, x, t)
    _, g16 = M.loss_and_grad(p, x, t, emulate=True)
    assert np.linalg.norm(g16 - g64) < 0.05 * np.linalg.norm(g64)
