"""FP64 oracle of the learned proposal network (first guesses that seed the
genetic algorithm's initial population, Sec. 5.5; neural-network inversion as
cited in Sec. 1).

TEST INFRASTRUCTURE ONLY, like the rest of this package: plain numpy in
float64, written from the definitions (affine layers, the erf form of GELU,
the squared-error loss, the chain rule, Adam), no blocking or fusion.

Conventions shared with the device library through the documented interface
only (no code is shared):
  * parameters are one flat vector, layer by layer W_l [out][in] then b_l [out];
  * hidden layers apply GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2,
    the output layer is affine;
  * features are the Stokes samples [4][L] divided by the pixel's maximum of I;
  * targets are the parameters scaled to [0, 1] by the search box; the loss is
    mean over the batch of sum_j d_j^2, d = y - t, with d of the azimuth
    (j = 2) taken to the nearest integer's remainder, the azimuth's period;
  * Adam with beta1 0.9, beta2 0.999, eps 1e-8 and bias correction.
The `bf16` switch rounds every matrix-product operand (inputs, weights,
hidden activations, back-propagated errors) to bfloat16, nearest-even, as the
device's matrix-core path stores them; accumulation stays in float64.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

DIMS = (1024, 512, 512, 512, 9)
AZIMUTH = 2


def layout(dims=DIMS):
    """[(w_offset, b_offset, n_out, n_in)] per layer and the total count."""
    out, o = [], 0
    for i in range(len(dims) - 1):
        nin, nout = dims[i], dims[i + 1]
        out.append((o, o + nout * nin, nout, nin))
        o += nout * nin + nout
    return out, o


def unpack(params, dims=DIMS):
    lay, n = layout(dims)
    params = np.asarray(params, np.float64)
    assert params.shape == (n,)
    return [(params[w:b].reshape(nout, nin), params[b:b + nout]) for w, b, nout, nin in lay]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, x, dims=DIMS, round_bf16=False):
    """Outputs y [n][dims[-1]] and the cache (layer inputs, pre-activations)."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    layers = unpack(params, dims)
    h = r(x)
    inputs, pres = [], []
    for li, (W, b) in enumerate(layers):
        inputs.append(h)
        z = h @ r(W).T + b
        pres.append(z)
        if li < len(layers) - 1:
            h = r(gelu(z))
    return z, dict(inputs=inputs, pres=pres)


def loss(y, target):
    """Loss and dL/dy."""
    d = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    d[:, AZIMUTH] -= np.rint(d[:, AZIMUTH])
    n = d.shape[0]
    return float((d * d).sum() / n), 2.0 * d / n


def backward(params, cache, dy, dims=DIMS, round_bf16=False):
    """Gradient of the loss with respect to every parameter (flat, float64)."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    layers = unpack(params, dims)
    lay, n = layout(dims)
    grad = np.empty(n)
    d = dy
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        w_off, b_off, nout, nin = lay[li]
        grad[w_off:b_off] = (r(d).T @ cache["inputs"][li]).ravel()
        grad[b_off:b_off + nout] = d.sum(axis=0)
        if li > 0:
            d = (r(d) @ r(W)) * gelu_prime(cache["pres"][li - 1])
    return grad


def loss_and_grad(params, x, target, dims=DIMS, round_bf16=False):
    y, cache = forward(params, x, dims, round_bf16)
    L, dy = loss(y, target)
    return L, backward(params, cache, dy, dims, round_bf16)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(obs):
    """obs [n][4][L] -> x [n][4 L], divided by each pixel's maximum of I."""
    obs = np.asarray(obs, np.float64)
    return (obs / obs[:, 0, :].max(axis=1)[:, None, None]).reshape(obs.shape[0], -1)


def scale(params, lo, hi):
    """Parameters -> targets in [0, 1] by the box."""
    return (np.asarray(params, np.float64) - lo) / (np.asarray(hi) - lo)


def unscale(y, lo, hi):
    """Network outputs -> parameters in the box (azimuth wrapped, then clamped)."""
    u = np.array(y, np.float64)
    u[:, AZIMUTH] -= np.floor(u[:, AZIMUTH])
    return np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * np.clip(u, 0.0, 1.0)
