"""Seeding generation 0 with first guesses (Sec. 5.5), through the C ABI:
bit-exact with the oracle's seeded initial population, the fused loop equal
to the step-by-step composition when seeded, and the service equal to a
standalone seeded inversion."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"


def _guesses(npix, seed):
    """First guesses inside the box, plus some outside it (clamped) and on its
    corners, as float32."""
    p = si.draw_uniform_box(npix, seed)
    p[0] = si.PRIOR_LO
    p[1] = si.PRIOR_HI
    if npix > 2:
        p[2] = si.PRIOR_LO - 0.3 * (si.PRIOR_HI - si.PRIOR_LO)
    if npix > 3:
        p[3] = si.PRIOR_HI + 0.3 * (si.PRIOR_HI - si.PRIOR_LO)
    return p.astype(np.float32)


@pytest.mark.parametrize("n_seeded,jitter", [(1, 0), (20, 37), (70, 1), (32, 32767)])
def test_seeded_ga_init_bit_exact(n_seeded, jitter):
    npix, pop = 6, 70
    sp = _guesses(npix, 3)
    cfg = g.GAConfig(pop=pop, seed=(5 << 32) | 17, pixel_base=1000, n_seeded=n_seeded,
                     seed_jitter=jitter, seed_params=torch.tensor(sp, device=DEV))
    got = g.ga_init(npix, cfg, g.bounds(si.PRIOR_LO, si.PRIOR_HI)).cpu().numpy()
    for p in range(npix):
        ref = oracle.ga_init(cfg.seed, 1000 + p, pop, n_seeded, jitter, sp[p].astype(np.float64),
                             si.PRIOR_LO, si.PRIOR_HI)
        assert np.array_equal(got[p], ref), p


def _problem(npix, seed):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set("slit"):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    truth = si.draw_truth(npix, seed)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return (lines, grids, olines, truth, torch.tensor(obs.astype(np.float32), device=DEV),
            torch.tensor(sig.astype(np.float32), device=DEV))


def test_seeded_fused_loop_equals_stepwise():
    lines, grids, olines, truth, obs, sig = _problem(9, 11)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    guess = torch.tensor((truth + 0.05 * (si.PRIOR_HI - si.PRIOR_LO)).astype(np.float32),
                         device=DEV)
    cfg = g.GAConfig(pop=64, generations=5, seed=4, pixel_base=2, n_seeded=16, seed_jitter=300,
                     seed_params=guess)
    fused = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    genes = g.ga_init(obs.shape[0], cfg, b)
    fit = g.ga_evaluate(genes, b, obs, sig, lines, grids)
    for t in range(1, cfg.generations + 1):
        genes = g.ga_step(genes, fit, cfg, t, diagnostics=False)["genes"]
        fit = g.ga_evaluate(genes, b, obs, sig, lines, grids)
    assert torch.equal(fused["genes"], genes)
    assert torch.equal(fused["fitness"], fit)
    # generation 0 of the fused loop is the oracle's seeded population
    cfg0 = g.GAConfig(**{**cfg.__dict__, "generations": 0})
    r0 = g.ga_invert(obs, sig, lines, grids, b, cfg0, want_population=True)
    gp = guess.cpu().numpy().astype(np.float64)
    for p in range(obs.shape[0]):
        ref = oracle.ga_init(4, 2 + p, 64, 16, 300, gp[p], si.PRIOR_LO, si.PRIOR_HI)
        assert np.array_equal(r0["genes"][p].cpu().numpy(), ref)


def test_seeding_with_truth_lowers_generation_zero_chi2():
    lines, grids, olines, truth, obs, sig = _problem(32, 12)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    kw = dict(pop=128, generations=0, seed=1)
    rand = g.ga_invert(obs, sig, lines, grids, b, g.GAConfig(**kw))
    seeded = g.ga_invert(obs, sig, lines, grids, b,
                         g.GAConfig(n_seeded=32, seed_jitter=64,
                                    seed_params=torch.tensor(truth.astype(np.float32), device=DEV),
                                    **kw))
    c0, c1 = rand["chi2"].cpu().numpy(), seeded["chi2"].cpu().numpy()
    assert np.all(c1 < 2.0)
    assert np.median(c0) > 20 * np.median(c1)


def test_serving_seeded_request_equals_ga_invert():
    lines, grids, olines, truth, obs, sig = _problem(50, 13)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    guess = torch.tensor(truth.astype(np.float32), device=DEV)
    cfg = g.GAConfig(pop=128, generations=17, seed=8, n_seeded=32, seed_jitter=500,
                     seed_params=guess)
    alone = g.ga_invert(obs, sig, lines, grids, b, cfg)
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=5)
    rid = sess.submit(obs, sig, lines, grids, b, cfg)
    for _ in range(20):
        if sess.poll(rid):
            break
        sess.step()
        torch.cuda.synchronize()
    assert sess.poll(rid) == 1
    out = sess.result(rid)
    assert torch.equal(out["params"], alone["params"])
    assert torch.equal(out["chi2"], alone["chi2"])
    sess.close()
