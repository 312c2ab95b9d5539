"""FP64 reference of the warm-start network: forward pass, mean-squared-error
gradient by the chain rule, and one Adam update.

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check.  The product
path never imports it; it shares no code with the HIP kernels.

The network (not in the paper; it predicts the cycle-averaged profiles the
paper computes in section 3, densities and mean energies across the gap):
  inputs  (U / U_max, normalised log p, x / L)
  4 hidden layers of 256 units, GELU with the exact error function
  6 outputs (log densities of e, O-, O2+ and their mean energies, standardised)
  loss    mean over the batch and the 6 outputs of (y - t)^2
  Adam    beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected, FP32 master
          weights in the product (FP64 here).

Parameter order in the flat vector: W0 (256 x 3), b0, W1 (256 x 256), b1, W2,
b2, W3, b3, W4 (6 x 256), b4; W_l[o, i] multiplies input i of output o.

With emulate=True the forward and backward round the quantities the product
holds in bfloat16 to bfloat16 (round to nearest even): the input x, every
weight matrix, every hidden activation, and the output and hidden-unit
gradients that enter a product.  Sums stay in FP64 (the product sums exact
bf16 x bf16 products in FP32), biases and pre-activations stay unrounded.
"""
from __future__ import annotations

import math

import numpy as np

SIZES = ((256, 3), (256, 256), (256, 256), (256, 256), (6, 256))
NPARAM = sum(o * i + o for o, i in SIZES)
_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def unflatten(p):
    """Views (W, b) of each layer in the flat parameter vector."""
    out, k = [], 0
    for o, i in SIZES:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    return out


def bf16(a):
    """Round FP32-representable values to bfloat16 (nearest, ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    """z Phi(z), Phi the standard normal distribution function."""
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_prime(z):
    """Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) * _INV_SQRT_2PI


def forward(p, x, emulate=False):
    """Returns the outputs y (B x 6) and the per-layer cache (input, pre-activation)."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    cache = []
    layers = unflatten(np.asarray(p, dtype=np.float64))
    for l, (W, b) in enumerate(layers):
        z = a @ r(W).T + b
        cache.append((a, z))
        a = r(gelu(z)) if l + 1 < len(layers) else z
    return a, cache


def loss_and_grad(p, x, t, emulate=False):
    """Mean squared error and its gradient with respect to the flat parameters."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    y, cache = forward(p, x, emulate)
    B = y.shape[0]
    diff = y - t
    loss = float(np.mean(diff * diff))
    layers = unflatten(np.asarray(p, dtype=np.float64))
    grads = [None] * len(layers)
    dz = 2.0 * diff / (B * y.shape[1])           # d loss / d z of the output layer
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in, _ = cache[l]
        dzr = r(dz)
        grads[l] = (dzr.T @ a_in, dz.sum(axis=0))
        if l > 0:
            da = dzr @ r(W)
            dz = da * gelu_prime(cache[l - 1][1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (step counts from 1); returns new p, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (seeded data
    for both sides)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for o, i in SIZES:
        s = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-s, s, size=o * i))
        parts.append(rng.uniform(-s, s, size=o))
    return np.concatenate(parts)
