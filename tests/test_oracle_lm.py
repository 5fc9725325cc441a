"""Pins of the oracle's FP64 Levenberg-Marquardt refinement: it never raises
chi-square, it converges to the noise-free truth from a nearby start, the
gradient of chi-square (by central differences of the oracle's merit function)
vanishes at its result, and on noisy data it beats the truth's chi-square."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _lines(kind):
    out = []
    for line, n in si.line_set(kind):
        st, sp = si.grid(line, n)
        out.append(oracle.make_line(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"],
                                    st, sp, n))
    return out


def _start(truth, seed, scale=0.01):
    rng = np.random.default_rng(seed)
    return np.clip(truth + (HI - LO) * rng.normal(0, scale, truth.shape), LO, HI)


def test_linearised_synthesis_at_the_base_point_is_the_synthesis():
    lines = _lines("slit")
    for p in si.draw_truth(4, 8):
        assert np.array_equal(oracle.me_synth_lin(p, p, lines, mu=0.7),
                              oracle.me_synth(p[None], lines, mu=0.7)[0])


@pytest.mark.parametrize("k", [0, 3, 4, 5])
def test_linearised_synthesis_error_is_second_order(k):
    # w(z0 + dz) - (w(z0) + w'(z0) dz) is O(dz^2): halving the step quarters
    # the error, and the error is a small fraction of the first-order change
    # (a wrong sign or constant in w', or v and a swapped, leaves an O(dz) error)
    lines = _lines("slit")
    for p0 in si.draw_truth(3, 9):
        errs = []
        for frac in (2e-3, 1e-3):
            p = p0.copy()
            p[k] = p0[k] + frac * (HI[k] - LO[k])
            exact = oracle.me_synth(p[None], lines)[0]
            lin = oracle.me_synth_lin(p0, p, lines)
            change = np.abs(exact - oracle.me_synth(p0[None], lines)[0]).max()
            err = np.abs(lin - exact).max()
            assert err <= 0.05 * change
            errs.append(err)
        assert 3.0 <= errs[0] / errs[1] <= 5.0, errs


def test_refine_never_increases_chi2_and_iteration_zero_is_identity():
    lines = _lines("tiny")
    truth = si.draw_truth(6, 1)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 1)
    p0 = _start(truth, 2, 0.05)
    c0 = oracle.chi2(p0[:, None], obs, sig, lines)[:, 0]
    prev = c0
    for it in (0, 1, 3, 10):
        r = oracle.lm_refine(obs, sig, lines, LO, HI, p0, it)
        assert np.all(r["chi2"] <= prev * (1 + 1e-12))
        prev = r["chi2"]
        if it == 0:
            assert np.allclose(r["params"], p0, rtol=0, atol=1e-12 * (HI - LO).max())
            assert np.allclose(r["chi2"], c0, rtol=1e-12)


def test_refine_converges_to_noise_free_truth():
    lines = _lines("slit")
    truth = si.draw_truth(6, 4)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    r = oracle.lm_refine(obs, sig, lines, LO, HI, _start(truth, 5), 60)
    err = np.abs(r["params"] - truth) / (HI - LO)
    ok = r["chi2"] < 1e-12
    assert ok.sum() >= 5
    # the field angles are undefined for weak fields: compare them only for B >= 100 G
    angles = np.zeros_like(err, dtype=bool)
    angles[:, 1:3] = truth[:, :1] < 100.0
    assert np.all(err[ok][~angles[ok]] < 1e-6)


def test_refine_gradient_vanishes_and_beats_truth_on_noisy_data():
    lines = _lines("tiny")
    truth = si.draw_truth(4, 7)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 7)
    r = oracle.lm_refine(obs, sig, lines, LO, HI, _start(truth, 8, 0.002), 100)
    ct = oracle.chi2(truth[:, None], obs, sig, lines)[:, 0]
    assert np.all(r["chi2"] <= ct)
    # central-difference gradient of chi2 in normalised coordinates at the result
    for p in range(4):
        x = (r["params"][p] - LO) / (HI - LO)
        grad = []
        for j in range(9):
            h = 1e-5
            if x[j] - h < 0 or x[j] + h > 1:
                continue                     # at a bound the gradient need not vanish
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            cp = oracle.chi2((LO + (HI - LO) * xp)[None, None], obs[p:p + 1], sig[p:p + 1], lines)[0, 0]
            cm = oracle.chi2((LO + (HI - LO) * xm)[None, None], obs[p:p + 1], sig[p:p + 1], lines)[0, 0]
            grad.append((cp - cm) / (2 * h))
        # compare with the curvature scale: |grad| << chi2 / (typical step)
        assert np.max(np.abs(grad)) < 1e-2 * max(r["chi2"][p], 1.0) / 1e-3


def test_refine_bad_pixels_and_bad_arguments():
    lines = _lines("tiny")
    truth = si.draw_truth(3, 9)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs[1, 0, 0] = np.nan
    r = oracle.lm_refine(obs, sig, lines, LO, HI, truth, 5)
    assert np.isnan(r["chi2"][1]) and np.isfinite(r["chi2"][[0, 2]]).all()
    with pytest.raises(ValueError):
        oracle.lm_refine(obs, sig, lines, LO, LO, truth, 5)
