"""The learned proposal network on the GPU, through the C ABI, against the FP64
oracle (oracle/mlp.py): forward and gradient in the FP32 mode and in the
BF16 matrix-core mode (the oracle then rounds the same operands), Adam, the
feature and scaling maps, the example generators, and a short training run
whose first guesses speed up the genetic algorithm (Sec. 5.5 seeding)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
import synth_inputs as si
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"
LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _slit():
    lines, grids, olines = [], [], []
    for ln, n in si.line_set("slit"):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    return lines, grids, olines


def _net(seed=3):
    net = g.MLP(seed=seed)
    return net, net.master.cpu().numpy().astype(np.float64)


def _x(n, seed):
    """Inputs shaped like real features: I near 1, Q, U, V small."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 0.05, size=(n, 1024))
    x[:, :256] += 0.8
    return x.astype(np.float32)


def test_init_statistics():
    net, p = _net(11)
    assert p.size == g.lib().mlp_param_count() == 1_054_729
    lay, _ = omlp.layout()
    for w, b, nout, nin in lay:
        W = p[w:b]
        assert np.all(p[b:b + nout] == 0.0)
        std = np.sqrt(2.0 / nin)
        assert abs(W.mean()) < 5 * std / np.sqrt(W.size)
        assert abs(W.std() / std - 1) < 5 * np.sqrt(0.5 / W.size) + 1e-3
    # a different seed gives different weights, the same seed the same
    assert not np.array_equal(p, _net(12)[1])
    assert np.array_equal(p, _net(11)[1])


@pytest.mark.parametrize("n", [1, 63, 300])
def test_forward_fp32_matches_oracle(n):
    net, p = _net()
    x = _x(n, n)
    y = net.forward(torch.tensor(x, device=DEV), precision=1).cpu().numpy()
    ref, _ = omlp.forward(p, x.astype(np.float64))
    scale = np.sqrt((ref ** 2).mean())
    assert np.abs(y - ref).max() <= 1e-5 * scale


@pytest.mark.parametrize("n", [5, 200])
def test_forward_bf16_matrix_cores(n):
    net, p = _net()
    x = _x(n, 100 + n)
    y = net.forward(torch.tensor(x, device=DEV), precision=0).cpu().numpy()
    emu, _ = omlp.forward(p, x.astype(np.float64), round_bf16=True)
    exact, _ = omlp.forward(p, x.astype(np.float64))
    scale = np.sqrt((exact ** 2).mean())
    # same rounded operands: only the FP32 accumulation order differs, and an
    # activation that this moves across a bfloat16 rounding boundary.  One such
    # flip shifts the next layer's inputs by a fraction of a bfloat16 step,
    # which re-rounds a few percent of them, so a row with an early flip ends
    # ~1e-2 relative away; rows without one agree to FP32 accuracy.
    row = np.abs(y - emu).max(axis=1)
    assert np.median(row) <= 1e-4 * scale
    assert np.linalg.norm(y - emu) <= 5e-3 * np.linalg.norm(emu)
    # and the BF16 network is the FP64 one to bfloat16 precision
    assert np.linalg.norm(y - exact) <= 2 ** -6 * np.linalg.norm(exact)


def _layer_errors(got, ref):
    lay, _ = omlp.layout()
    out = []
    for w, b, nout, nin in lay:
        for a, c in ((w, b), (b, b + nout)):
            out.append(np.linalg.norm(got[a:c] - ref[a:c]) / np.linalg.norm(ref[a:c]))
    return np.array(out)


@pytest.mark.parametrize("batch", [7, 130])
def test_gradient_fp32_matches_oracle(batch):
    net, p = _net(5)
    x = _x(batch, 7 * batch)
    t = np.random.default_rng(batch).uniform(size=(batch, 9)).astype(np.float32)
    grad, loss = net.compute_grad(torch.tensor(x, device=DEV), torch.tensor(t, device=DEV),
                                  precision=1)
    L, gref = omlp.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - L) <= 1e-5 * L
    assert np.all(_layer_errors(grad.cpu().numpy().astype(np.float64), gref) <= 1e-4)


# 1000: the weight gradients split the batch into eight k ranges, the last
# ragged; 4096: the training batch (a full round of 128-row tiles)
@pytest.mark.parametrize("batch", [1, 9, 256, 1000, 4096])
def test_gradient_bf16_matches_oracle(batch):
    net, p = _net(6)
    x = _x(batch, 3 * batch)
    t = np.random.default_rng(batch + 1).uniform(size=(batch, 9)).astype(np.float32)
    grad, loss = net.compute_grad(torch.tensor(x, device=DEV), torch.tensor(t, device=DEV),
                                  precision=0)
    got = grad.cpu().numpy().astype(np.float64)
    Le, gemu = omlp.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64),
                                  round_bf16=True)
    L, gref = omlp.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - Le) <= 1e-4 * Le
    assert np.all(_layer_errors(got, gemu) <= 5e-3)
    assert np.all(_layer_errors(got, gref) <= 3e-2)


def test_adam_matches_oracle():
    net, p = _net(7)
    rng = np.random.default_rng(1)
    g1 = rng.normal(0, 1e-2, p.size).astype(np.float32)
    g2 = rng.normal(0, 1e-2, p.size).astype(np.float32)
    pm, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for step, gr in ((1, g1), (2, g2), (3, g1)):
        net.grad.copy_(torch.tensor(gr, device=DEV))
        net.adam(3e-4)
        pm, m, v = omlp.adam(pm, m, v, gr.astype(np.float64), step, 3e-4)
    got = net.master.cpu().numpy()
    assert np.abs(got - pm).max() <= 1e-6 * np.abs(pm).max() + 3e-4 * 1e-4
    # the moments mix gradients of both signs, so compare at FP32 resolution
    # of their scale rather than element-relative
    for got_m, ref_m in ((net.m, m), (net.v, v)):
        got_m = got_m.cpu().numpy()
        assert np.abs(got_m - ref_m).max() <= 1e-6 * np.abs(ref_m).max()


def test_features_and_unscale_match_oracle():
    lines, grids, olines = _slit()
    truth = si.draw_truth(40, 2)
    obs = oracle.me_synth(truth, olines).astype(np.float32)
    net = g.MLP(seed=0)
    x = net.features(torch.tensor(obs, device=DEV), grids).cpu().numpy()
    assert np.allclose(x, omlp.features(obs.astype(np.float64)), rtol=3e-7, atol=0)
    y = np.random.default_rng(4).uniform(-0.3, 1.3, size=(40, 9)).astype(np.float32)
    params = torch.empty((40, 9), dtype=torch.float32, device=DEV)
    b = g.bounds(LO, HI)
    import ctypes as C
    g._check(g.lib().mlp_unscale(g._ptr(torch.tensor(y, device=DEV)), 40, C.byref(b),
                                 g._ptr(params), None))
    torch.cuda.synchronize()
    ref = omlp.unscale(y.astype(np.float64), LO, HI)
    assert np.allclose(params.cpu().numpy(), ref, rtol=1e-6, atol=1e-6 * (HI - LO).max())


def _philox_words(seed, c0, c1, c2, c3):
    return oracle.philox4x32_10([c0, c1, c2, c3], [seed & 0xFFFFFFFF, seed >> 32])


def _box_muller(w0, w1):
    u1 = ((int(w0) >> 8) + 1) / 16777217.0
    u2 = (int(w1) >> 8) / 16777216.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def test_example_generators_follow_their_streams():
    lines, grids, olines = _slit()
    seed, first, n = (3 << 32) | 5, 1000, 24
    net = g.MLP(seed=0)
    b = g.bounds(LO, HI)
    params = torch.empty((n, 9), dtype=torch.float32, device=DEV)
    target = torch.empty_like(params)
    import ctypes as C
    g._check(g.lib().mlp_draw_examples(seed, first, n, C.byref(b), g._ptr(params),
                                       g._ptr(target), None))
    torch.cuda.synchronize()
    P, T = params.cpu().numpy(), target.cpu().numpy()
    for i in range(n):
        gi = first + i
        ws = np.concatenate([_philox_words(seed, gi & 0xFFFFFFFF, gi >> 32, 1, (7 << 24) | k)
                             for k in range(3)])
        u = (ws[:9] >> 8).astype(np.float64) / 16777216.0
        z = _box_muller(ws[9], ws[10])
        u[3] = min(max(0.5 + 0.1 * z, 0.0), 1.0)
        keep = np.arange(9) != 3
        assert np.array_equal(T[i, keep], u[keep].astype(np.float32))
        assert np.array_equal(P[i, keep], (LO + (HI - LO) * u)[keep].astype(np.float32))
        assert abs(T[i, 3] - u[3]) <= 1e-6
    # noise: sigma_rel (S0 + S1) times the normal of word pair (e, purpose 8)
    clean = g.me_synth(params, lines, grids)
    noisy = clean.clone()
    ga = (g.MeGrid * 2)(*grids)
    g._check(g.lib().mlp_add_noise(seed, first, g._ptr(params), n, ga, 2, 1e-3, g._ptr(noisy),
                                   None))
    torch.cuda.synchronize()
    d = (noisy - clean).cpu().numpy().reshape(n, -1)
    for i in (0, 7, n - 1):
        gi = first + i
        ic = float(P[i, 7]) + float(P[i, 8])
        for e in (0, 1, 300, 1023):
            w = _philox_words(seed, gi & 0xFFFFFFFF, gi >> 32, 2, (8 << 24) | e)
            assert abs(d[i, e] - 1e-3 * ic * _box_muller(w[0], w[1])) <= 2e-7 * max(ic, 1.0)


def test_train_loop_equals_its_steps():
    # one mlp_train call of 3 steps = the same steps through the separate
    # entry points (draw, synthesise, noise, features, gradient, Adam)
    lines, grids, olines = _slit()
    b = g.bounds(LO, HI)
    a = g.MLP(seed=9)
    losses = a.train(lines, grids, b, steps=3, batch=64, lr=1e-3, seed=17).cpu().numpy()
    c = g.MLP(seed=9)
    for s in range(3):
        x, t = c.examples(17, s * 64, 64, lines, grids, b, sigma_rel=1e-3)
        _, loss = c.compute_grad(x, t)
        assert loss.item() == losses[s]
        c.adam(1e-3)
    assert torch.equal(a.master, c.master)


def test_training_learns_and_seeding_speeds_up_the_search():
    lines, grids, olines = _slit()
    b = g.bounds(LO, HI)
    net = g.MLP(seed=1)
    first = net.train(lines, grids, b, steps=50, batch=512, lr=1e-3, seed=2).cpu().numpy()
    net.train(lines, grids, b, steps=1450, batch=512, lr=1e-3, seed=2)
    last = net.train(lines, grids, b, steps=100, batch=512, lr=3e-4, seed=2).cpu().numpy()
    assert np.isfinite(last).all()
    assert last.mean() < 0.25 * first[:10].mean()
    # held-out pixels (a different generator) with the benchmark's noise
    truth = si.draw_truth(256, 77)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = (obs + sig[:, :, None] * si.std_normal(obs.shape, 77)).astype(np.float32)
    obs_t = torch.tensor(obs, device=DEV)
    sig_t = torch.tensor(sig.astype(np.float32), device=DEV)
    guess = net.predict(obs_t, grids, b)
    # the proposal is informative: its field strength beats the prior's spread
    err_b = np.abs(guess[:, 0].cpu().numpy() - truth[:, 0])
    assert np.median(err_b) < 0.25 * np.median(np.abs(truth[:, 0] - 1500.0))
    kw = dict(pop=128, tournament_k=4, seed=4)
    for gens in (20, 60):
        r0 = g.ga_invert(obs_t, sig_t, lines, grids, b, g.GAConfig(generations=gens, **kw))
        r1 = g.ga_invert(obs_t, sig_t, lines, grids, b,
                         g.GAConfig(generations=gens, n_seeded=32, seed_jitter=512,
                                    seed_params=guess, **kw))
        c0, c1 = r0["chi2"].cpu().numpy(), r1["chi2"].cpu().numpy()
        assert np.median(c1) < 0.7 * np.median(c0), (gens, np.median(c0), np.median(c1))
