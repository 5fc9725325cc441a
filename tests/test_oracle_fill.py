"""Pins of the oracle's magnetic fill fraction (Sec. 5.2).

The field-free profile is pinned by closed forms: a depth of exactly d at the
line centre, the Gaussian 1 - d exp(-v^2) for zero damping (H(v, 0) =
exp(-v^2)), symmetry about the model's line centre and a continuum of 1 far
out.  The mixed Stokes vector reduces to the Milne-Eddington one at alpha = 1
and to the field-free one at alpha = 0.  The closed-form best alpha is pinned
against a brute-force scan of the chi-square built from the synthesis alone,
against the true alpha of noise-free observations, and at the clamps."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _lines(kind):
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set(kind)]


def _fill(kind, lo=0.0, hi=1.0):
    return oracle.make_fill(lo, hi, *si.fill_coefficients(kind))


def _centred_line(nlam=41, step=0.01):
    ln = si.FE6302
    return oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                            ln["lambda0"] - step * (nlam // 2), step, nlam)


def test_field_free_profile_closed_forms():
    line = _centred_line()
    fl = oracle.FillLine()
    for k, (d, w, a) in enumerate(zip((0.6, 0.0, 0.0, 0.0), (0.03, 0.0, 0.0, 0.0),
                                      (0.25, 0.0, 0.0, 0.0))):
        fl.depth[k], fl.width[k], fl.damp[k] = d, w, a
    N = oracle.fill_profile(line, fl, 1.0, 0.0)
    c = len(N) // 2
    # absolute wavelengths (6302 A) carry rounding of ~1e-12 A, i.e. ~3e-11
    # in v: the closed forms hold to 1e-9
    assert N[c] == pytest.approx(0.4, abs=1e-9)             # depth d at the centre
    assert np.allclose(N[:c][::-1], N[c + 1:], rtol=0, atol=1e-9)    # symmetric
    assert np.all(N <= 1.0) and np.all(N[c:-1] <= N[c + 1:])
    # zero damping: a Gaussian of 1/e half width w
    fl.damp[0] = 0.0
    N0 = oracle.fill_profile(line, fl, 1.0, 0.0)
    v = (np.arange(len(N0)) - c) * 0.01 / 0.03
    assert np.allclose(N0, 1.0 - 0.6 * np.exp(-v * v), rtol=0, atol=1e-9)
    # the centre follows the model velocity
    vl = 0.01 / si.FE6302["lambda0"] * 299792.458 * 3      # three samples redward
    Nv = oracle.fill_profile(line, fl, 1.0, vl)
    assert Nv[c + 3] == pytest.approx(0.4, abs=1e-9)
    # the polynomial in mu, and an invalid width
    fl.depth[1] = 0.2
    assert oracle.fill_profile(line, fl, 0.5, 0.0)[c] == pytest.approx(1.0 - 0.7, abs=1e-9)
    fl.width[1] = -0.05
    with pytest.raises(ValueError):
        oracle.fill_profile(line, fl, 1.0, 0.0)


def test_mixture_end_points():
    lines = _lines("slit")
    f = _fill("slit")
    p = si.draw_truth(5, 1)
    mu = np.linspace(0.3, 1.0, 5)
    m = oracle.me_synth(p, lines, mu=mu)
    assert np.array_equal(oracle.me_synth_fill(p, np.ones(5), lines, f, mu=mu), m)
    z = oracle.me_synth_fill(p, np.zeros(5), lines, f, mu=mu)
    assert np.all(z[:, 1:] == 0.0)
    off = 0
    for ln, fl in zip(lines, f.line):
        for i in range(5):
            N = oracle.fill_profile(ln, fl, mu[i], p[i, 3])
            ic = p[i, 7] + mu[i] * p[i, 8]
            assert np.allclose(z[i, 0, off:off + ln.nlam], ic * N, rtol=1e-15, atol=0)
        off += ln.nlam


def test_best_alpha_is_the_brute_force_minimum():
    lines = _lines("slit")
    f = _fill("slit")
    truth = si.draw_truth(4, 2)
    alpha = si.draw_alpha(4, 2)
    obs = oracle.me_synth_fill(truth, alpha, lines, f)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 2)
    # candidate models near (not at) the truth
    rng = np.random.default_rng(3)
    cand = np.clip(truth + (HI - LO) * rng.normal(0, 0.02, truth.shape), LO, HI)
    c, a = oracle.chi2_fill(cand[:, None], obs, sig, lines, f)
    L = obs.shape[-1]
    grid = np.linspace(0, 1, 2001)
    for i in range(4):
        scan = []
        for g in grid:
            mdl = oracle.me_synth_fill(cand[i:i + 1], [g], lines, f)[0]
            scan.append((((obs[i] - mdl) / sig[i][:, None]) ** 2).sum() / (4 * L - 10))
        scan = np.array(scan)
        assert abs(a[i, 0] - grid[np.argmin(scan)]) <= 1.0 / 2000 + 1e-12
        assert c[i, 0] <= scan.min() * (1 + 1e-12)
        assert c[i, 0] >= scan.min() * (1 - 1e-5)


def test_best_alpha_recovers_the_truth_and_clamps():
    lines = _lines("slit")
    truth = si.draw_truth(6, 4)
    alpha = si.draw_alpha(6, 4)
    f = _fill("slit")
    obs = oracle.me_synth_fill(truth, alpha, lines, f)
    sig = si.sigma_for(truth)
    c, a = oracle.chi2_fill(truth[:, None], obs, sig, lines, f)
    assert np.allclose(a[:, 0], alpha, rtol=0, atol=1e-10)
    assert np.all(c[:, 0] < 1e-12)
    # a range that excludes the truth: the nearest end
    lo = oracle.make_fill(0.9, 1.0, *si.fill_coefficients("slit"))
    c2, a2 = oracle.chi2_fill(truth[:, None], obs, sig, lines, lo)
    assert np.all(a2[:, 0] == np.maximum(alpha, 0.9))
    fixed = oracle.make_fill(1.0, 1.0, *si.fill_coefficients("slit"))
    c3, a3 = oracle.chi2_fill(truth[:, None], obs, sig, lines, fixed)
    assert np.all(a3 == 1.0)
    # alpha fixed at 1 is the plain merit function with one more degree of freedom used
    L = obs.shape[-1]
    plain = oracle.chi2(truth[:, None], obs, sig, lines)[:, 0]
    assert np.allclose(c3[:, 0] * (4 * L - 10), plain * (4 * L - 9), rtol=1e-12)


def test_ga_with_fill_uses_the_fill_merit():
    lines = _lines("tiny")
    f = _fill("tiny", 0.25, 1.0)
    truth = si.draw_truth(3, 5)
    alpha = si.draw_alpha(3, 5)
    obs = oracle.me_synth_fill(truth, alpha, lines, f)
    sig = si.sigma_for(truth)
    res = oracle.ga_invert(obs, sig, lines, LO, HI, pop=16, generations=4, k=4, p_cross=0.85,
                           p_mut=0.05, seed=2, fill=f, want_population=True)
    par = oracle.decode(res["genes"].reshape(-1, 9), LO, HI).reshape(3, 16, 9)
    c, a = oracle.chi2_fill(par, obs, sig, lines, f)
    assert np.array_equal(res["fitness"], c)
    best = np.argmin(c, axis=1)
    assert np.array_equal(res["alpha"], a[np.arange(3), best])
    assert np.all((res["alpha"] >= 0.25) & (res["alpha"] <= 1.0))
    # a width that is not positive at a pixel's mu: status 4
    bad = oracle.make_fill(0.25, 1.0, *si.fill_coefficients("tiny"))
    bad.line[0].width[1] = -0.05       # width 0.036 - 0.05 mu < 0 for mu > 0.72
    r = oracle.ga_invert(obs, sig, lines, LO, HI, pop=8, generations=1, k=2, p_cross=0.8,
                         p_mut=0.05, seed=1, fill=bad, mu=np.array([0.5, 0.9, 1.0]))
    assert list(r["status"]) == [0, 4, 4]
    assert np.isnan(r["alpha"][1]) and np.isfinite(r["alpha"][0])


# ---- the Levenberg-Marquardt fit with alpha as a tenth coordinate ---------

def _fill_problem(npix=6, seed=3, alpha=None, kind="tiny"):
    lines = _lines(kind)
    f = _fill(kind, 0.1, 1.0)
    truth = si.draw_truth(npix, seed)
    al = np.linspace(0.35, 0.9, npix) if alpha is None else np.full(npix, alpha)
    mu = np.linspace(0.45, 1.0, npix)
    obs = oracle.me_synth_fill(truth, al, lines, f, mu=mu)
    sig = si.sigma_for(truth, mu=mu)
    return lines, f, truth, al, mu, obs, sig


def test_fill_fit_with_alpha_held_at_one_is_the_plain_fit():
    # at alpha = 1 the fill model is the Milne-Eddington vector itself, so the
    # ten-coordinate fit with alpha held takes the plain fit's steps; only nu
    # (4L - 10 against 4L - 9) rescales its chi-square
    lines = _lines("tiny")
    f = _fill("tiny", 0.0, 1.0)
    truth = si.draw_truth(5, 8)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    start = np.clip(truth + 0.03 * (si.PRIOR_HI - si.PRIOR_LO), si.PRIOR_LO, si.PRIOR_HI)
    plain = oracle.lm_refine(obs, sig, lines, LO, HI, start, 6)
    fill = oracle.lm_refine_fill(obs, sig, lines, LO, HI, f, start, np.ones(5), 6,
                                 free_mask=0x1FF)
    assert np.array_equal(fill["params"], plain["params"])
    assert np.array_equal(fill["iters"], plain["iters"])
    assert np.all(fill["alpha"] == 1.0)
    L = sum(ln.nlam for ln in lines)
    assert np.allclose(fill["chi2"] * (4 * L - 10), plain["chi2"] * (4 * L - 9), rtol=1e-12,
                       atol=0)


def test_fill_fit_recovers_noise_free_truth():
    lines, f, truth, al, mu, obs, sig = _fill_problem()
    # start from the truth moved by 1 % of every range and alpha moved by 0.1
    start = np.clip(truth + 0.01 * (si.PRIOR_HI - si.PRIOR_LO), si.PRIOR_LO, si.PRIOR_HI)
    r = oracle.lm_refine_fill(obs, sig, lines, LO, HI, f, start, al - 0.1, 60, mu=mu)
    assert np.all(r["chi2"] < 1e-10), r["chi2"]
    assert np.allclose(r["alpha"], al, rtol=0, atol=1e-6)
    assert np.allclose(r["params"][:, 0], truth[:, 0], rtol=1e-5, atol=1e-3)
    # the chi-square of the result is the merit function of Sec. 5 at (p, alpha)
    m = oracle.me_synth_fill(r["params"], r["alpha"], lines, f, mu=mu)
    L = m.shape[2]
    direct = (((obs - m) / sig[:, :, None]) ** 2).sum(axis=(1, 2)) / (4 * L - 10)
    assert np.allclose(direct, r["chi2"], rtol=1e-9, atol=1e-300)


def test_fill_fit_alpha_is_stationary_at_the_closed_form_best():
    # with noise, the fitted alpha (interior) is where d chi2 / d alpha = 0 at
    # the fitted parameters: the closed-form best alpha of the GA's merit
    # (pinned above against a brute-force scan) at the same parameters
    lines, f, truth, al, mu, obs, sig = _fill_problem(npix=5, seed=11)
    rng = np.random.default_rng(4)
    noisy = obs + sig[:, :, None] * rng.standard_normal(obs.shape)
    start = np.clip(truth + 0.01 * (si.PRIOR_HI - si.PRIOR_LO), si.PRIOR_LO, si.PRIOR_HI)
    r = oracle.lm_refine_fill(noisy, sig, lines, LO, HI, f, start, al, 80, mu=mu)
    c_best, a_best = oracle.chi2_fill(r["params"][:, None, :], noisy, sig, lines, f, mu=mu)
    inner = (r["alpha"] > 0.1 + 1e-3) & (r["alpha"] < 1 - 1e-3)
    assert inner.sum() >= 4
    assert np.allclose(r["alpha"][inner], a_best[inner, 0], rtol=0, atol=2e-5)
    # and the fit's chi-square is that merit's minimum over alpha
    assert np.allclose(r["chi2"], c_best[:, 0], rtol=1e-7, atol=0)
    # the refinement never raises the chi-square of its start
    c0, _ = oracle.chi2_fill(start[:, None, :], noisy, sig, lines, f, mu=mu)
    m0 = oracle.me_synth_fill(start, al, lines, f, mu=mu)
    L = m0.shape[2]
    chi_start = (((noisy - m0) / sig[:, :, None]) ** 2).sum(axis=(1, 2)) / (4 * L - 10)
    assert np.all(r["chi2"] <= chi_start)


def test_fill_fit_bad_pixels_and_arguments():
    lines, f, truth, al, mu, obs, sig = _fill_problem(npix=3)
    obs = obs.copy()
    obs[1, 0, 4] = np.nan
    r = oracle.lm_refine_fill(obs, sig, lines, LO, HI, f, truth, al, 3, mu=mu)
    assert np.isnan(r["chi2"][1]) and np.isnan(r["alpha"][1]) and np.isnan(r["params"][1]).all()
    assert np.isfinite(r["chi2"][[0, 2]]).all()
    with pytest.raises(ValueError):
        oracle.lm_refine_fill(obs, sig, lines, LO, HI, _fill("tiny", 0.5, 0.5), truth, al, 3)
    with pytest.raises(ValueError):
        oracle.lm_refine_fill(obs, sig, lines, LO, HI, f, truth, al, -1)
