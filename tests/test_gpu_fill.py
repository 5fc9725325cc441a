"""Magnetic fill fraction (Sec. 5.2) through the C ABI, against the oracle.

Bars: the mixed Stokes vector within 1e-5 I_c (FP32, the forward model's bar)
and 1e-10 I_c (FP64); the FP64 loop on the oracle's trajectory (bit-exact
operators, near-ties aside) with its alpha and chi-square to 1e-9; the FP32
loop's fitness within the bound the forward-model tolerance implies for the
chi-square at the best alpha (the minimum over alpha moves only to second
order with the model), (1/nu) sum w^2 (2 |r| delta + delta^2)."""
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
LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _setup(kind):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set(kind):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    return lines, grids, olines


def _fills(kind, lo=0.0, hi=1.0):
    c = si.fill_coefficients(kind)
    return g.fill(lo, hi, *c), oracle.make_fill(lo, hi, *c)


def _t(x, dt):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


@pytest.mark.parametrize("dt,tol", [(torch.float32, 1e-5), (torch.float64, 1e-10)])
def test_synth_fill_matches_oracle(dt, tol):
    lines, grids, olines = _setup("slit")
    gf, of = _fills("slit")
    n = 300
    p = si.draw_uniform_box(n, 3)
    alpha = np.random.default_rng(4).uniform(0, 1, n)
    alpha[:10], alpha[10:20] = 0.0, 1.0
    mu = np.linspace(0.2, 1.0, n)
    npdt = np.float32 if dt == torch.float32 else np.float64
    p, alpha, mu = p.astype(npdt), alpha.astype(npdt), mu.astype(npdt)
    got = g.me_synth(_t(p, dt), lines, grids, mu=_t(mu, dt), alpha=_t(alpha, dt), fill=gf)
    ref = oracle.me_synth_fill(p.astype(np.float64), alpha.astype(np.float64), olines, of,
                               mu=mu.astype(np.float64))
    ic = (p[:, 7] + mu * p[:, 8]).astype(np.float64)[:, None, None]
    err = np.abs(got.cpu().numpy().astype(np.float64) - ref) / ic
    assert np.isfinite(err).all()
    assert err.max() <= tol, err.max()
    # invalid field-free profile at a model's mu: NaN rows, the others untouched
    bad_c = [np.array(a) for a in si.fill_coefficients("slit")]
    bad_c[1][:, 1] = -0.05
    gb = g.fill(0.0, 1.0, *bad_c)
    got2 = g.me_synth(_t(p, dt), lines, grids, mu=_t(mu, dt), alpha=_t(alpha, dt), fill=gb)
    w = bad_c[1][0, 0] + mu * (bad_c[1][0, 1] + mu * bad_c[1][0, 2])
    bad = w <= 0
    assert bad.any() and (~bad).any()
    g2 = got2.cpu().numpy().astype(np.float64)
    assert np.isnan(g2[bad]).all()
    ob = oracle.make_fill(0.0, 1.0, *bad_c)
    ref2 = oracle.me_synth_fill(p.astype(np.float64), alpha.astype(np.float64), olines, ob,
                                mu=mu.astype(np.float64))
    assert np.isnan(ref2[bad]).all()
    # near-zero widths divide the oracle's rounding of absolute wavelengths
    # (~1e-12 A) by w: scale the bar by 0.02 A / w there
    scale = np.maximum(1.0, 0.02 / np.where(bad, 1.0, w))[:, None, None]
    assert np.all((np.abs(g2[~bad] - ref2[~bad]) / ic[~bad]) <= tol * scale[~bad])


def _problem(kind, npix, seed, lo, hi):
    lines, grids, olines = _setup(kind)
    gf, of = _fills(kind, lo, hi)
    truth = si.draw_truth(npix, seed)
    alpha = si.draw_alpha(npix, seed)
    obs = oracle.me_synth_fill(truth, alpha, olines, of)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return lines, grids, olines, gf, of, truth, alpha, obs, sig


def test_fill_loop_f64_tracks_the_oracle():
    lines, grids, olines, gf, of, truth, alpha, obs, sig = _problem("tiny", 12, 31, 0.25, 1.0)
    cfg = g.GAConfig(pop=48, generations=10, tournament_k=4, seed=3, init_mode=1,
                     restart_every=4)
    r = g.ga_invert(_t(obs, torch.float64), _t(sig, torch.float64), lines, grids,
                    g.bounds(LO, HI), cfg, want_population=True, fill=gf)
    ref = oracle.ga_invert(obs, sig, olines, LO, HI, pop=48, generations=10, k=4,
                           p_cross=cfg.p_cross, p_mut=cfg.p_mut, seed=3, init_mode=1,
                           restart_every=4, want_population=True, fill=of)
    same = [np.array_equal(r["genes"][p].cpu().numpy(), ref["genes"][p]) for p in range(12)]
    # bit-exact operators; a fitness near-tie (1e-13 relative) may flip a decision
    assert sum(same) >= 10, same
    c, cr = r["chi2"].cpu().numpy(), ref["chi2"]
    a, ar = r["alpha"].cpu().numpy(), ref["alpha"]
    assert np.all(np.abs(c - cr)[same] <= 1e-9 * cr[same])
    assert np.all(np.abs(a - ar)[same] <= 1e-9)
    assert np.all((a >= 0.25) & (a <= 1.0))


def test_fill_loop_f32_fitness_is_the_fill_merit():
    lines, grids, olines, gf, of, truth, alpha, obs, sig = _problem("slit", 6, 32, 0.0, 1.0)
    cfg = g.GAConfig(pop=64, generations=8, seed=5)
    r = g.ga_invert(_t(obs, torch.float32), _t(sig, torch.float32), lines, grids,
                    g.bounds(LO, HI), cfg, want_population=True, fill=gf)
    genes = r["genes"].cpu().numpy()
    par = oracle.decode(genes.reshape(-1, 9), LO, HI).reshape(6, 64, 9)
    o32 = obs.astype(np.float32).astype(np.float64)
    s32 = sig.astype(np.float32).astype(np.float64)
    ref, aref = oracle.chi2_fill(par, o32, s32, olines, of)
    fit = r["fitness"].cpu().numpy().astype(np.float64)
    L = obs.shape[-1]
    models = np.stack([oracle.me_synth_fill(par[p], aref[p], olines, of) for p in range(6)])
    ic = (par[..., 7] + par[..., 8])[..., None, None]
    delta = 1e-5 * ic
    rr = np.abs(o32[:, None] - models)
    w2 = 1.0 / s32[:, None, :, None] ** 2
    bound = (w2 * (2 * rr * delta + delta ** 2)).sum(axis=(2, 3)) / (4 * L - 10)
    assert np.all(np.abs(fit - ref) <= bound + 1e-5 * ref)
    e = np.argmin(fit, axis=1)
    assert np.array_equal(r["chi2"].cpu().numpy(), fit[np.arange(6), e].astype(np.float32))
    da = np.abs(r["alpha"].cpu().numpy() - aref[np.arange(6), e])
    assert np.median(da) <= 1e-5 and da.max() <= 1e-3, da


def test_fill_loop_fp16_fitness_is_its_fill_merit():
    # FP16 profile synthesis with the fill fraction: every final fitness is the
    # fill merit (closed-form best alpha) of me_synth_f16's Stokes vector of
    # the decoded genes, and within the FP16 synthesis bound (5e-3 Ic per
    # sample) of the oracle's fill merit
    lines, grids, olines, gf, of, truth, alpha, obs, sig = _problem("slit", 6, 35, 0.1, 1.0)
    cfg = g.GAConfig(pop=64, generations=6, seed=7, synth_precision=g.SYNTH_FP16)
    r = g.ga_invert(_t(obs, torch.float32), _t(sig, torch.float32), lines, grids,
                    g.bounds(LO, HI), cfg, want_population=True, fill=gf)
    genes = r["genes"].cpu().numpy()
    par = oracle.decode(genes.reshape(-1, 9), LO, HI)
    M = g.me_synth(torch.tensor(par, dtype=torch.float32, device=DEV), lines, grids,
                   fp16=True).cpu().numpy().astype(np.float64).reshape(6, 64, 4, -1)
    L = M.shape[-1]
    N = np.stack([np.concatenate([oracle.fill_profile(ln, fl, 1.0, p[3])
                                  for ln, fl in zip(olines, of.line)]) for p in par])
    N = N.reshape(6, 64, L)
    ic = (par[:, 7] + par[:, 8]).reshape(6, 64, 1)
    o = obs.astype(np.float32).astype(np.float64)[:, None]
    w2 = 1.0 / sig.astype(np.float32).astype(np.float64)[:, None, :, None] ** 2
    bvec = np.zeros_like(M)
    bvec[:, :, 0] = ic * N
    D, e = M - bvec, o - M
    see, sed, sdd = ((w2 * e * e).sum(axis=(2, 3)), (w2 * e * D).sum(axis=(2, 3)),
                     (w2 * D * D).sum(axis=(2, 3)))
    beta = np.clip(-sed / sdd, 1.0 - of.alpha_hi, 1.0 - of.alpha_lo)
    merit = (see + beta * (2 * sed + beta * sdd)) / (4 * L - 10)
    fit = r["fitness"].cpu().numpy().astype(np.float64)
    assert np.allclose(fit, merit, rtol=1e-3, atol=0)
    e_best = np.argmin(fit, axis=1)
    da = np.abs(r["alpha"].cpu().numpy() - (1.0 - beta)[np.arange(6), e_best])
    assert da.max() <= 1e-3, da
    # against the FP64 oracle's fill merit of the same genes
    ref, aref = oracle.chi2_fill(par.reshape(6, 64, 9), o[:, 0], np.sqrt(1.0 / w2[:, 0, :, 0]),
                                 olines, of)
    models = np.stack([oracle.me_synth_fill(par.reshape(6, 64, 9)[q], aref[q], olines, of)
                       for q in range(6)])
    delta = 5e-3 * ic[..., None]
    rr = np.abs(o - models)
    bound = (w2 * (2 * rr * delta + delta ** 2)).sum(axis=(2, 3)) / (4 * L - 10)
    assert np.all(np.abs(fit - ref) <= bound + 1e-5 * ref)


def test_fill_status_and_rejections():
    lines, grids, olines, gf, of, truth, alpha, obs, sig = _problem("slit", 4, 33, 0.0, 1.0)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    b = g.bounds(LO, HI)
    bad_c = [np.array(a) for a in si.fill_coefficients("slit")]
    bad_c[1][:, 1] = -0.05          # width <= 0 for mu > 0.72
    mu = _t(np.array([0.5, 0.6, 0.9, 1.0]), torch.float32)
    r = g.ga_invert(o32, s32, lines, grids, b, g.GAConfig(pop=16, generations=2),
                    mu=mu, fill=g.fill(0.0, 1.0, *bad_c))
    assert r["status"].cpu().tolist() == [0, 0, 4, 4]
    assert torch.isnan(r["alpha"][2:]).all() and torch.isfinite(r["alpha"][:2]).all()
    with pytest.raises(g.GenesisError):
        g.ga_invert(_t(obs, torch.float64), _t(sig, torch.float64), lines, grids, b,
                    g.GAConfig(pop=16, generations=2, synth_precision=g.SYNTH_FP16), fill=gf)
    with pytest.raises(g.GenesisError):
        g.ga_invert(o32, s32, lines, grids, b, g.GAConfig(pop=16, generations=2),
                    fill=g.fill(0.5, 0.2, *si.fill_coefficients("slit")))


def test_alpha_fixed_at_one_is_the_plain_merit():
    lines, grids, olines, gf, of, truth, alpha, obs, sig = _problem("slit", 5, 34, 1.0, 1.0)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    cfg = g.GAConfig(pop=64, generations=0, seed=9)
    one = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg, want_population=True,
                      fill=gf)
    plain = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg, want_population=True)
    assert torch.equal(one["genes"], plain["genes"])
    assert torch.all(one["alpha"] == 1.0)
    L = obs.shape[-1]
    f1 = one["fitness"].cpu().numpy().astype(np.float64) * (4 * L - 10)
    f0 = plain["fitness"].cpu().numpy().astype(np.float64) * (4 * L - 9)
    assert np.allclose(f1, f0, rtol=2e-5, atol=0)


# ---- FP64 Levenberg-Marquardt refinement of the fill model ----------------

def _fill_refine_problem(npix, seed, noise, kind="slit"):
    lines, grids, olines = _setup(kind)
    gf, of = _fills(kind, 0.1, 1.0)
    truth = si.draw_truth(npix, seed)
    al = np.linspace(0.3, 0.95, npix)
    mu = np.linspace(0.4, 1.0, npix)
    obs = oracle.me_synth_fill(truth, al, olines, of, mu=mu)
    sig = si.sigma_for(truth, mu=mu)
    if noise:
        obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed + 1)
    rng = np.random.default_rng(seed + 2)
    p0 = np.clip(truth + (HI - LO) * rng.normal(0, 0.01, truth.shape), LO, HI)
    a0 = np.clip(al + rng.normal(0, 0.05, npix), 0.1, 1.0)
    return lines, grids, olines, gf, of, truth, al, mu, obs, sig, p0, a0


@pytest.mark.parametrize("noise", [False, True])
def test_refine_fill_matches_oracle(noise):
    # both fits reach the same minimum of the fill model's chi-square (the
    # FP64 models differ by < 1e-10 I_c, the Gram matrices by rounding order)
    (lines, grids, olines, gf, of, truth, al, mu, obs, sig, p0,
     a0) = _fill_refine_problem(10, 21, noise)
    f64 = torch.float64
    r = g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, g.bounds(LO, HI), gf,
                             _t(p0, f64), _t(a0, f64), iterations=40, mu=_t(mu, f64))
    ref = oracle.lm_refine_fill(obs, sig, olines, LO, HI, of, p0, a0, 40, mu=mu)
    gp, ga, gc = (r[k].cpu().numpy() for k in ("params", "alpha", "chi2"))
    dx = np.abs(gp - ref["params"]) / (HI - LO)
    same = (dx.max(axis=1) < 1e-6) & (np.abs(ga - ref["alpha"]) < 1e-6)
    print("pixels at the oracle's minimum: %d / 10" % same.sum())
    assert same.sum() >= 9
    assert np.all(np.abs(gc[same] - ref["chi2"][same])
                  <= 1e-7 * np.maximum(ref["chi2"][same], 1e-6))
    # the reported chi-square is the oracle's merit at the returned (p, alpha)
    m = oracle.me_synth_fill(gp, ga, olines, of, mu=mu)
    L = m.shape[2]
    direct = (((obs - m) / sig[:, :, None]) ** 2).sum(axis=(1, 2)) / (4 * L - 10)
    assert np.allclose(gc, direct, rtol=1e-9, atol=1e-14)
    if not noise:
        ok = gc < 1e-12
        assert ok.sum() >= 8
        assert np.all(np.abs(ga[ok] - al[ok]) < 1e-6)


def test_refine_fill_with_alpha_held_at_one_is_the_plain_refinement():
    # at alpha = 1 the fill model is the Milne-Eddington vector, so holding
    # alpha (bit 9 clear) gives the plain refinement's parameters to the bit
    lines, grids, olines = _setup("slit")
    gf, of = _fills("slit", 0.0, 1.0)
    truth = si.draw_truth(16, 5)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    rng = np.random.default_rng(6)
    p0 = np.clip(truth + (HI - LO) * rng.normal(0, 0.01, truth.shape), LO, HI)
    f64 = torch.float64
    b = g.bounds(LO, HI)
    plain = g.me_refine_f64(_t(obs, f64), _t(sig, f64), lines, grids, b, _t(p0, f64), 12)
    fill = g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, b, gf, _t(p0, f64),
                                _t(np.ones(16), f64), iterations=12, free_mask=0x1FF)
    assert torch.equal(fill["params"], plain["params"])
    assert torch.equal(fill["iters"], plain["iters"])
    assert torch.all(fill["alpha"] == 1.0)
    L = sum(gr.n for gr in grids)
    assert torch.allclose(fill["chi2"] * (4 * L - 10), plain["chi2"] * (4 * L - 9), rtol=1e-12,
                          atol=0)


def test_refine_fill_edge_cases():
    (lines, grids, olines, gf, of, truth, al, mu, obs, sig, p0,
     a0) = _fill_refine_problem(4, 8, False, kind="tiny")
    obs = obs.copy()
    obs[1, 2, 3] = np.nan
    f64 = torch.float64
    b = g.bounds(LO, HI)
    a0 = a0.copy()
    a0[2] = 7.0                            # outside [alpha_lo, alpha_hi]: clamped
    r = g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, b, gf, _t(truth, f64),
                             _t(a0, f64), iterations=0, mu=_t(mu, f64))
    assert np.isnan(r["params"][1].cpu().numpy()).all() and np.isnan(r["alpha"][1].item())
    assert r["alpha"][2].item() == pytest.approx(1.0, abs=1e-12)
    assert int(r["iters"][0].item()) == 0
    # a field-free profile invalid at this mu: NaN, like a bad observation
    bad_c = [np.array(a) for a in si.fill_coefficients("tiny")]
    bad_c[1][0][0] = -1.0                  # width(mu) < 0 everywhere
    bad = g.fill(0.1, 1.0, *bad_c)
    r = g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, b, bad, _t(truth, f64),
                             _t(a0, f64), iterations=2, mu=_t(mu, f64))
    assert torch.isnan(r["chi2"]).all()
    # arguments
    with pytest.raises(g.GenesisError):
        g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, b,
                             g.fill(0.5, 0.5, *si.fill_coefficients("tiny")), _t(truth, f64),
                             _t(a0, f64), iterations=2, mu=_t(mu, f64))
    empty = g.me_refine_fill_f64(_t(obs[:0], f64), _t(sig[:0], f64), lines, grids, b, gf,
                                 _t(truth[:0], f64), _t(a0[:0], f64), iterations=3)
    assert empty["params"].shape == (0, 9)


def test_ga_fill_then_refine_fill_pipeline():
    # the FP32 fill-fraction search followed by the FP64 fill refinement on
    # noise-free observations: the refinement lowers every chi-square and
    # brings alpha and B closer to the truth
    lines, grids, olines = _setup("slit")
    gf, of = _fills("slit", 0.1, 1.0)
    npix = 128
    truth = si.draw_truth(npix, 30)
    al = np.linspace(0.3, 0.95, npix)
    obs = oracle.me_synth_fill(truth, al, olines, of)
    sig = si.sigma_for(truth)
    b = g.bounds(LO, HI)
    ga = g.ga_invert(_t(obs, torch.float32), _t(sig, torch.float32), lines, grids, b,
                     g.GAConfig(pop=128, generations=120, seed=3), fill=gf)
    f64 = torch.float64
    r = g.me_refine_fill_f64(_t(obs, f64), _t(sig, f64), lines, grids, b, gf,
                             ga["params"].double(), ga["alpha"].double(), iterations=30)
    c_ga = ga["chi2"].double().cpu().numpy()
    c_r = r["chi2"].cpu().numpy()
    assert np.all(c_r <= c_ga * 1.001 + 1e-6)
    e_ga = np.abs(ga["alpha"].double().cpu().numpy() - al)
    e_r = np.abs(r["alpha"].cpu().numpy() - al)
    print("median |d alpha| GA %.3g, GA + refine %.3g" % (np.median(e_ga), np.median(e_r)))
    assert np.median(e_r) < np.median(e_ga)
