"""Pins of the FP64 proposal-network oracle (oracle/mlp.py).

The hand-written chain rule is pinned against central finite differences and
against an independent differentiation (torch autograd in float64 on the CPU);
GELU, the wrapped loss, Adam's first step, bfloat16 rounding and the feature
and scaling maps against closed forms and special cases.
"""
import numpy as np
import pytest
import torch

from oracle import mlp
import synth_inputs as si

TINY = (12, 6, 6, 6, 9)


def _params(dims, seed, scale=0.6):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mlp.layout(dims)[1])


def test_layout_matches_documented_count():
    lay, n = mlp.layout()
    assert n == 1024 * 512 + 512 + 2 * (512 * 512 + 512) + 512 * 9 + 9 == 1_054_729
    assert lay[0] == (0, 1024 * 512, 512, 1024)
    assert lay[-1][1] + 9 == n


def test_gelu_identities():
    x = np.linspace(-6, 6, 241)
    # x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x)) = x
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, rtol=0, atol=1e-15)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-20 and abs(mlp.gelu(-10.0)) < 1e-20
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_prime(x), fd, rtol=0, atol=1e-9)
    assert mlp.gelu_prime(0.0) == 0.5


def test_bf16_rounding_special_cases():
    one = 1.0
    cases = {one: one, one + 2 ** -8: one, one + 3 * 2 ** -8: one + 2 ** -6,
             one + 2 ** -7: one + 2 ** -7, -2.5: -2.5, 0.0: 0.0}
    for x, want in cases.items():
        assert mlp.bf16(np.array([x]))[0] == want, x
    # agrees with torch's own nearest-even conversion on random values
    v = np.random.default_rng(0).normal(0, 10, 10000)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(v), ref)


def test_loss_wraps_azimuth():
    y = np.zeros((1, 9))
    t = np.zeros((1, 9))
    y[0, 2], t[0, 2] = 0.05, 0.95
    L, dy = mlp.loss(y, t)
    assert abs(L - 0.01) < 1e-15 and abs(dy[0, 2] - 0.2) < 1e-15
    # a full period in the azimuth output changes nothing; other outputs do
    y2 = y.copy()
    y2[0, 2] += 1.0
    assert abs(mlp.loss(y2, t)[0] - L) < 1e-15
    y3 = y.copy()
    y3[0, 0] = 1.0
    assert abs(mlp.loss(y3, t)[0] - (L + 1.0)) < 1e-15


def test_zero_weights_closed_form():
    # every weight zero: y = b_out for every input, and the only nonzero
    # gradients are those of the output bias, 2 mean(y - t)
    dims = TINY
    p = np.zeros(mlp.layout(dims)[1])
    lay, n = mlp.layout(dims)
    b_out = np.arange(9) / 10.0
    p[lay[-1][1]:] = b_out
    rng = np.random.default_rng(3)
    x = rng.normal(size=(5, 12))
    t = rng.uniform(size=(5, 9)) * 0.3
    y, _ = mlp.forward(p, x, dims)
    assert np.array_equal(y, np.tile(b_out, (5, 1)))
    L, g = mlp.loss_and_grad(p, x, t, dims)
    gb = g[lay[-1][1]:]
    assert np.allclose(gb, 2 * (b_out - t).mean(axis=0), rtol=0, atol=1e-15)
    # hidden biases see zero downstream weights; the last weight matrix sees
    # activations gelu(0) = 0
    assert np.all(g[:lay[-1][1]] == 0.0)


def test_gradient_matches_finite_differences():
    dims = TINY
    p = _params(dims, 1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(7, 12))
    t = rng.uniform(size=(7, 9))
    L, g = mlp.loss_and_grad(p, x, t, dims)
    idx = rng.choice(p.size, 60, replace=False)
    lay, _ = mlp.layout(dims)
    idx = np.concatenate([idx, [lay[i][1] for i in range(4)]])   # a bias of every layer
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, t, dims)[0] - mlp.loss_and_grad(pm, x, t, dims)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_matches_autograd_full_size():
    p = _params(mlp.DIMS, 4, scale=0.04)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4, 1024))
    t = rng.uniform(size=(4, 9))
    L, g = mlp.loss_and_grad(p, x, t)
    # independent differentiation of the same definition
    P = torch.tensor(p, requires_grad=True)
    X, T = torch.tensor(x), torch.tensor(t)
    h = X
    lay, _ = mlp.layout()
    for li, (w, b, nout, nin) in enumerate(lay):
        W = P[w:b].reshape(nout, nin)
        z = h @ W.T + P[b:b + nout]
        h = z * 0.5 * (1 + torch.erf(z / np.sqrt(2))) if li < 3 else z
    d = h - T
    d = torch.cat([d[:, :2], (d[:, 2] - torch.round(d[:, 2]).detach())[:, None], d[:, 3:]], 1)
    Lt = (d * d).sum() / 4
    Lt.backward()
    assert abs(Lt.item() - L) <= 1e-12 * L
    ref = P.grad.numpy()
    assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()


def test_bf16_mode_is_close_to_exact():
    # rounding the operands moves the loss and gradient only at bfloat16's
    # relative precision (2^-8)
    p = _params(mlp.DIMS, 6, scale=0.04)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(8, 1024))
    t = rng.uniform(size=(8, 9))
    L, g = mlp.loss_and_grad(p, x, t)
    Lb, gb = mlp.loss_and_grad(p, x, t, round_bf16=True)
    assert abs(Lb - L) <= 2 ** -6 * L
    assert np.linalg.norm(gb - g) <= 2 ** -5 * np.linalg.norm(g)
    assert np.linalg.norm(gb - g) > 0


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2: the step is -lr g / (|g| + eps)
    rng = np.random.default_rng(8)
    g = rng.normal(size=100)
    p0 = rng.normal(size=100)
    p1, m, v = mlp.adam(p0, np.zeros(100), np.zeros(100), g, 1, 1e-3)
    assert np.allclose(p1 - p0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    p, m, v = p0, np.zeros(100), np.zeros(100)
    for s in range(1, 6):
        q, m, v = mlp.adam(p, m, v, g, s, 1e-3)
        assert np.allclose(q - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=0)
        p = q


def test_features_and_scaling():
    rng = np.random.default_rng(9)
    obs = rng.uniform(0.1, 1.0, size=(3, 4, 256))
    x = mlp.features(obs)
    assert x.shape == (3, 1024)
    assert np.allclose(x[:, :256].max(axis=1), 1.0)
    assert np.allclose(mlp.features(obs * 7.5), x, rtol=1e-15)
    p = si.draw_uniform_box(50, 3)
    t = mlp.scale(p, si.PRIOR_LO, si.PRIOR_HI)
    assert t.min() >= 0 and t.max() <= 1
    assert np.allclose(mlp.unscale(t, si.PRIOR_LO, si.PRIOR_HI), p, rtol=1e-14, atol=1e-12)
    # out-of-range outputs clamp to the box, the azimuth wraps
    y = np.full((1, 9), 1.25)
    q = mlp.unscale(y, si.PRIOR_LO, si.PRIOR_HI)
    assert np.allclose(np.delete(q[0], 2), np.delete(si.PRIOR_HI, 2))
    assert abs(q[0, 2] - 0.25 * 180.0) < 1e-12
