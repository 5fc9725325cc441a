"""GPU FP64 Levenberg-Marquardt refinement against the oracle's refinement and
the noise-free truth."""
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


def _start(truth, seed, scale):
    rng = np.random.default_rng(seed)
    return np.clip(truth + (HI - LO) * rng.normal(0, scale, truth.shape), LO, HI)


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("noise", [False, True])
def test_refine_matches_oracle(noise):
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(10, 12)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    if noise:
        obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 12)
    p0 = _start(truth, 13, 0.01)
    b = g.bounds(LO, HI)
    r = g.me_refine_f64(_t(obs), _t(sig), lines, grids, b, _t(p0), iterations=40)
    ref = oracle.lm_refine(obs, sig, olines, LO, HI, p0, 40)
    gp = r["params"].cpu().numpy()
    gc = r["chi2"].cpu().numpy()
    dx = np.abs(gp - ref["params"]) / (HI - LO)
    # both converge to the same minimum (FP64 models differ by < 1e-10 Ic)
    same = dx.max(axis=1) < 1e-6
    print("pixels at the oracle's minimum: %d / 10" % same.sum())
    assert same.sum() >= 9
    assert np.all(np.abs(gc[same] - ref["chi2"][same]) <= 1e-7 * np.maximum(ref["chi2"][same], 1e-6))
    # never worse than the start
    c0 = oracle.chi2(p0[:, None], obs, sig, olines)[:, 0]
    assert np.all(gc <= c0 * (1 + 1e-9))
    if not noise:
        ok = gc < 1e-12
        assert ok.sum() >= 8
        err = np.abs(gp - truth) / (HI - LO)
        angles = np.zeros_like(err, dtype=bool)
        angles[:, 1:3] = truth[:, :1] < 100.0
        assert np.all(err[ok][~angles[ok]] < 1e-6)


@pytest.mark.parametrize("iterations", [1, 3])
def test_refine_iterates_follow_the_oracle(iterations):
    # the same steps as the oracle (reading 20, linearised Jacobian columns
    # included), not only the same minimum: after 1 and 3 iterations from a
    # distant start the parameters equal the oracle's to 1e-4 of the step taken
    # (the two FP64 models differ by ~1e-13, which the h = 1e-7 differences
    # turn into ~1e-6 relative differences of the Jacobian)
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(10, 21)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 21)
    p0 = _start(truth, 22, 0.05)
    r = g.me_refine_f64(_t(obs), _t(sig), lines, grids, g.bounds(LO, HI), _t(p0),
                        iterations=iterations)
    ref = oracle.lm_refine(obs, sig, olines, LO, HI, p0, iterations)
    gp = r["params"].cpu().numpy()
    step = np.abs(ref["params"] - p0).max(axis=1) / (HI - LO).max()
    dx = (np.abs(gp - ref["params"]) / (HI - LO)).max(axis=1)
    close = dx <= 1e-4 * step + 1e-9
    print("iterations %d: pixels on the oracle's iterate %d / 10, max dx / step %.2e"
          % (iterations, close.sum(), (dx / np.maximum(step, 1e-30)).max()))
    assert close.sum() >= 9


def test_refine_edge_cases():
    lines, grids, olines = _setup("tiny")
    truth = si.draw_truth(4, 3)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs[2, 1, 4] = np.inf
    b = g.bounds(LO, HI)
    p0 = truth.copy()
    p0[0, 0] = 5000.0                        # outside the box: clamped
    r = g.me_refine_f64(_t(obs), _t(sig), lines, grids, b, _t(p0), iterations=0)
    gp = r["params"].cpu().numpy()
    assert np.isnan(gp[2]).all() and np.isnan(r["chi2"][2].item())
    assert abs(gp[0, 0] - HI[0]) < 1e-9
    keep = [1, 3]
    assert np.allclose(gp[keep], truth[keep], rtol=1e-12, atol=1e-12)
    empty = g.me_refine_f64(_t(obs[:0]), _t(sig[:0]), lines, grids, b, _t(p0[:0]), 5)
    assert empty["params"].shape == (0, 9)


def test_ga_then_refine_pipeline_reaches_truth():
    """The FP32 genetic search followed by the FP64 refinement on noise-free
    synthetic truth of the slit-row line pair."""
    lines, grids, olines = _setup("slit")
    npix = 256
    truth = si.draw_truth(npix, 0)
    tt = torch.tensor(truth, dtype=torch.float32, device=DEV)
    obs = g.me_synth(tt, lines, grids)
    sig = torch.tensor(si.sigma_for(truth), dtype=torch.float32, device=DEV)
    b = g.bounds(LO, HI)
    ga = g.ga_invert(obs, sig, lines, grids, b, g.GAConfig(pop=128, generations=200, seed=0))
    r = g.me_refine_f64(obs.double(), sig.double(), lines, grids, b, ga["params"].double(), 50)
    dB_ga = np.abs(ga["params"][:, 0].double().cpu().numpy() - truth[:, 0])
    dB = np.abs(r["params"][:, 0].cpu().numpy() - truth[:, 0])
    print("p50/p90 |dB| GA %.2f / %.2f G, GA+refine %.3g / %.3g G"
          % (np.median(dB_ga), np.percentile(dB_ga, 90), np.median(dB), np.percentile(dB, 90)))
    assert np.median(dB) < np.median(dB_ga)
    assert np.all(r["chi2"].cpu().numpy() <= ga["chi2"].double().cpu().numpy() * 1.001 + 1e-6)


def _noisy(olines, n, seed, strong=True):
    truth = si.draw_truth(n, seed)
    if strong:
        truth[:, 0] = np.linspace(600.0, 2800.0, n)
        truth[:, 5] = np.clip(truth[:, 5], 0.05, 0.45)
        truth[:, 7] = np.clip(truth[:, 7], 0.05, 0.45)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return truth, obs, sig


def test_uncertainties_match_oracle():
    """Sec. 6 uncertainties: the GA's final population gives the initial
    steps (ga_population_steps, bit-exact with the oracle's), the oracle's
    refined optimum is the point, and the device's Hessian (Jacobian of the
    Richardson-extrapolated gradient) must agree with the oracle's within
    their tableaux' error estimates plus 1e-6 of the curvature scale (the two
    FP64 merit functions differ by ~1e-8 absolute, smoothly in p, so the
    tableaux take the same path), and sigma to 2e-3 (the inverse amplifies H's
    differences by its condition number)."""
    lines, grids, olines = _setup("slit")
    n = 6
    truth, obs, sig = _noisy(olines, n, 14)
    b = g.bounds(LO, HI)
    o32 = torch.tensor(obs, dtype=torch.float32, device=DEV)
    s32 = torch.tensor(sig, dtype=torch.float32, device=DEV)
    ga = g.ga_invert(o32, s32, lines, grids, b, g.GAConfig(pop=64, generations=60, seed=3),
                     want_population=True)
    ref = oracle.lm_refine(obs, sig, olines, LO, HI, truth, 40)
    popt = ref["params"]
    steps = g.ga_population_steps(ga["genes"], ga["fitness"], b, _t(popt)).cpu().numpy()
    genes = ga["genes"].cpu().numpy()
    fit = ga["fitness"].double().cpu().numpy()
    assert np.array_equal(steps, oracle.population_steps(genes, fit, LO, HI, popt))
    u = g.me_uncertainty_f64(_t(obs), _t(sig), lines, grids, b, _t(popt), _t(steps),
                             want_hessian=True)
    uo = oracle.uncertainty(obs, sig, olines, LO, HI, popt, steps)
    assert np.array_equal(u["steps"].cpu().numpy(), uo["steps"])
    H = u["hessian"].cpu().numpy()
    He = u["hessian_err"].cpu().numpy()
    for p in range(n):
        d = np.abs(H[p] - uo["hess"][p])
        scale = np.sqrt(np.abs(np.outer(np.diag(uo["hess"][p]), np.diag(uo["hess"][p]))))
        print("pixel %d: max |dH| / scale %.2e, / (err) %.2e" % (
            p, np.max(d / scale), np.max(d / (He[p] + uo["hess_err"][p] + 1e-300))))
        assert np.all(d <= 20 * (He[p] + uo["hess_err"][p]) + 1e-6 * scale)
    gs = u["sigma"].cpu().numpy()
    ok = np.isfinite(uo["sigma"])
    assert np.array_equal(np.isfinite(gs), ok)
    assert np.all(np.abs(gs[ok] - uo["sigma"][ok]) <= 2e-3 * uo["sigma"][ok])
    print("max sigma rel diff %.2e" % np.max(np.abs(gs[ok] - uo["sigma"][ok]) / uo["sigma"][ok]))


def test_uncertainty_edge_cases_match_oracle():
    """Held parameters (free_mask), a parameter at its bound, a bad pixel and
    huge or zero initial steps: the same NaN pattern, steps and (within the
    bound above) values as the oracle."""
    lines, grids, olines = _setup("tiny")
    truth, obs, sig = _noisy(olines, 4, 15)
    truth[1, 5] = LO[5]
    obs[2, 3, 7] = np.nan
    steps = np.tile(0.01 * (HI - LO), (4, 1))
    steps[3] = 1e9
    steps[0, 4] = 0.0
    b = g.bounds(LO, HI)
    mask = 0x1FF & ~(1 << 2) & ~(1 << 7)
    u = g.me_uncertainty_f64(_t(obs), _t(sig), lines, grids, b, _t(truth), _t(steps),
                             free_mask=mask, want_hessian=True)
    uo = oracle.uncertainty(obs, sig, olines, LO, HI, truth, steps, free_mask=mask)
    assert np.array_equal(u["steps"].cpu().numpy(), uo["steps"])
    gs = u["sigma"].cpu().numpy()
    assert np.array_equal(np.isnan(gs), np.isnan(uo["sigma"]))
    assert np.isnan(gs[2]).all() and np.isnan(gs[:, [2, 7]]).all() and np.isnan(gs[1, 5])
    ok = np.isfinite(uo["sigma"])
    assert np.all(np.abs(gs[ok] - uo["sigma"][ok]) <= 2e-3 * uo["sigma"][ok])
    with pytest.raises(g.GenesisError):
        g.me_uncertainty_f64(_t(obs), _t(sig), lines, grids, b, _t(truth), _t(steps),
                             free_mask=0)
    e = g.me_uncertainty_f64(_t(obs[:0]), _t(sig[:0]), lines, grids, b, _t(truth[:0]),
                             _t(steps[:0]))
    assert e["sigma"].shape == (0, 9)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_population_steps_bit_exact(dtype):
    rng = np.random.default_rng(7)
    for pop in (1, 2, 5, 64, 128, 1024):
        npix = 3
        genes = rng.integers(0, 65536, size=(npix, pop, 9)).astype(np.uint16)
        fit = rng.uniform(1, 3, size=(npix, pop))
        if pop >= 8:
            fit[0, 3] = np.nan
            fit[1, 2] = fit[1, 6] = fit[1].min() - 1.0
        fit = fit.astype(np.float32 if dtype == torch.float32 else np.float64)
        popt = rng.uniform(LO, HI, size=(npix, 9))
        b = g.bounds(LO, HI)
        got = g.ga_population_steps(torch.tensor(genes.view(np.int16), device=DEV).view(torch.uint16),
                                    torch.tensor(fit, device=DEV), b, _t(popt)).cpu().numpy()
        ref = oracle.population_steps(genes, fit.astype(np.float64), LO, HI, popt)
        assert np.array_equal(got, ref), pop


def test_uncertainties_of_a_long_observation_are_invariant_to_replicating_the_line():
    """Scale invariance of Sec. 6's sigma at an observation too long to stage
    in LDS: repeating the line's samples k times multiplies the reduced merit
    function by c = k (4L - 9) / (4kL - 9), so H and chi2(p_opt) scale by c
    and sigma^2 = [H^-1]_jj chi2 / M does not change."""
    ln = si.FE6302
    n, k = 1200, 4
    st, sp = si.grid(ln, n)
    line = g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"])
    oline = oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"], st, sp, n)
    truth, obs, sig = _noisy([oline], 3, 21)
    steps = np.tile(0.01 * (HI - LO), (3, 1))
    b = g.bounds(LO, HI)
    one = g.me_uncertainty_f64(_t(obs), _t(sig), [line], [g.grid(st, sp, n)], b, _t(truth),
                               _t(steps), want_hessian=True)
    obs_k = np.concatenate([obs] * k, axis=2)
    rep = g.me_uncertainty_f64(_t(obs_k), _t(sig), [line] * k, [g.grid(st, sp, n)] * k, b,
                               _t(truth), _t(steps), want_hessian=True)
    c = k * (4.0 * n - 9) / (4.0 * k * n - 9)
    s1, sk = one["sigma"].cpu().numpy(), rep["sigma"].cpu().numpy()
    assert np.array_equal(np.isfinite(s1), np.isfinite(sk))
    ok = np.isfinite(s1)
    assert ok.sum() >= 20
    assert np.all(np.abs(sk[ok] - s1[ok]) <= 1e-3 * s1[ok])
    H1, Hk = one["hessian"].cpu().numpy(), rep["hessian"].cpu().numpy()
    for p in range(3):
        d = np.abs(np.diag(H1[p]))
        scale = np.sqrt(np.outer(d, d))
        assert np.all(np.abs(Hk[p] - c * H1[p]) <= 1e-4 * scale + 1e-300)
