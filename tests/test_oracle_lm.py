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


# ---- uncertainties (Sec. 6) ---------------------------------------------------

def _tiny_lines():
    import synth_inputs as si
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set("tiny")]


def _strong_truth(n, seed):
    import synth_inputs as si
    t = si.draw_truth(n, seed)
    t[:, 0] = 1200.0 + 600.0 * np.arange(n) / max(n - 1, 1)
    t[:, 1] = 35.0 + 10.0 * np.arange(n) % 90
    t[:, 6] = 8.0
    return t


def test_uncertainty_matches_finite_difference_hessian():
    """sigma_j^2 = [H^-1]_jj chi2 / M with H the Hessian of the reduced
    chi-square: the oracle's Gauss-Newton H against a central-difference
    Hessian of the chi-square itself, at the optimum of noisy data (the two
    differ only by the residual-weighted curvature, a few per cent)."""
    import synth_inputs as si
    lines = _tiny_lines()
    truth = _strong_truth(3, 8)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 8)
    r = oracle.lm_refine(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, truth, 60)
    span = si.PRIOR_HI - si.PRIOR_LO
    M = 9
    for p in range(3):
        p0 = r["params"][p]
        h = 2e-4 * span

        def chi(q):
            return oracle.chi2(q[None, None, :], obs[p:p + 1], sig[p:p + 1], lines)[0, 0]

        H = np.empty((M, M))
        for a in range(M):
            for b in range(M):
                ea = np.eye(M)[a] * h[a]
                eb = np.eye(M)[b] * h[b]
                H[a, b] = (chi(p0 + ea + eb) - chi(p0 + ea - eb) - chi(p0 - ea + eb)
                           + chi(p0 - ea - eb)) / (4 * h[a] * h[b])
        sfd = np.sqrt(np.diag(np.linalg.inv(H)) * r["chi2"][p] / M)
        rel = np.abs(r["sigma"][p] - sfd) / sfd
        assert np.all(np.isfinite(r["sigma"][p])) and np.all(r["sigma"][p] > 0)
        assert np.all(rel < 0.15), rel


def test_uncertainty_tracks_the_scatter_of_repeated_inversions():
    """Monte Carlo: the textbook covariance (J_p^T J_p)^-1 that the formula
    scales by (nu/2)(chi2/M) matches the scatter of refined parameters over
    independent noise draws."""
    import synth_inputs as si
    lines = _tiny_lines()
    truth = np.repeat(_strong_truth(1, 9), 120, axis=0)
    clean = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = clean + sig[:, :, None] * si.std_normal(clean.shape, 19)
    r = oracle.lm_refine(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, truth, 60)
    nu = 4 * 100 - 9
    textbook = r["sigma"] * np.sqrt(2 * 9 / (nu * r["chi2"][:, None]))
    pred = np.median(textbook, axis=0)
    spread = r["params"].std(axis=0)
    for j in (0, 1, 3, 4, 6):      # B, inclination, v_los, Doppler width, eta0
        assert 0.75 < spread[j] / pred[j] < 1.33, (j, spread[j], pred[j])
