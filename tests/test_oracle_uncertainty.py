"""Pins of the oracle's Sec. 6 uncertainties (oracle/oracle_unc.c): the Hessian
as the Jacobian of a Richardson-extrapolated gradient, the variances
sigma_j^2 = [H^-1]_jj chi2 / M, and the initial steps from the final
population.

What fixes them without an implementation to compare against:
 * analytic functions with known Hessians (quadratic, quartic, exponential
   and trigonometric terms) reproduced to 1e-8 or better;
 * closed forms of the variance formula (diagonal H, held parameters, a
   parameter the function ignores, an indefinite H);
 * on the Milne-Eddington merit function at noise-free truth the exact
   Hessian equals its Gauss-Newton form (2/nu) J^T J (the residual term
   vanishes), with J from the oracle's forward model by plain central
   differences, not the tableaux;
 * two different initial steps give the same Hessian within the tableaux'
   own error estimates;
 * the scatter of independent noisy inversions matches the textbook
   covariance that the paper's formula scales by (nu / 2)(chi2 / M);
 * hand-built populations give the stated RMS over the stated ranks.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

LO, HI = si.PRIOR_LO, si.PRIOR_HI
SPAN = HI - LO


def _lines(kind):
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set(kind)]


# ---- the derivative machinery on analytic functions ----------------------

def test_hessian_of_quadratic_and_quartic():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(9, 9))
    A = A @ A.T + 9 * np.eye(9)
    a4 = rng.uniform(0.5, 2.0, 9)
    Bc = rng.normal(size=(9, 9)) * 0.3
    np.fill_diagonal(Bc, 0.0)
    b = rng.normal(size=9)

    def f(x):
        return 0.5 * x @ A @ x + b @ x + np.sum(a4 * x ** 4) + np.sum(Bc * np.outer(x ** 2, x))

    def hess(x):
        H = A + np.diag(12 * a4 * x ** 2)
        # sum_ij B_ij x_i^2 x_j: d2/dx_k^2 = 2 sum_j B_kj x_j; d2/dx_k dx_l = 2 B_kl x_k + 2 B_lk x_l
        H += np.diag(2 * Bc @ x)
        off = 2 * (Bc * x[:, None]) + 2 * (Bc.T * x[None, :])
        np.fill_diagonal(off, 0.0)
        return H + off

    x = rng.uniform(-1, 1, 9)
    H, He = oracle.sec6_hessian(f, x, np.full(9, 0.3))
    ref = hess(x)
    assert np.max(np.abs(H - ref)) <= 1e-8 * np.max(np.abs(ref))
    assert np.allclose(H, H.T, rtol=0, atol=0)
    # pure quadratic: exact to rounding
    Hq, _ = oracle.sec6_hessian(lambda x: 0.5 * x @ A @ x + b @ x, x, np.full(9, 0.5))
    assert np.max(np.abs(Hq - A)) <= 1e-12 * np.max(np.abs(A))


def test_hessian_of_transcendental_function():
    rng = np.random.default_rng(2)
    u = rng.normal(size=6) * 0.5
    v = rng.normal(size=6) * 0.7

    def f(x):
        return np.exp(u @ x) + np.sin(v @ x) + np.log1p(x[0] ** 2)

    def hess(x):
        H = np.exp(u @ x) * np.outer(u, u) - np.sin(v @ x) * np.outer(v, v)
        H[0, 0] += (2 - 2 * x[0] ** 2) / (1 + x[0] ** 2) ** 2
        return H

    x = rng.uniform(-0.5, 0.5, 6)
    H, He = oracle.sec6_hessian(f, x, rng.uniform(0.05, 0.4, 6))
    ref = hess(x)
    assert np.max(np.abs(H - ref)) <= 1e-8 * np.max(np.abs(ref))
    # the error estimates are honest: the true error is within a few of them
    assert np.all(np.abs(H - ref) <= 10 * He + 1e-13 * np.max(np.abs(ref)))


def test_hessian_active_mask_and_plain_step_fails_without_extrapolation():
    A = np.diag(np.arange(1.0, 6.0))

    def f(x):
        return 0.5 * x @ A @ x + np.cos(x[0]) * x[1] ** 3

    x = np.array([0.3, -0.2, 0.5, 0.1, 0.7])
    act = np.array([1, 1, 0, 1, 0], np.int32)
    H, He = oracle.sec6_hessian(f, x, np.full(5, 0.4), act)
    assert np.all(H[2] == 0) and np.all(H[:, 4] == 0)
    ref = A.copy()
    ref[0, 0] += -np.cos(x[0]) * x[1] ** 3
    ref[1, 1] += 6 * np.cos(x[0]) * x[1]
    ref[0, 1] = ref[1, 0] = -np.sin(x[0]) * 3 * x[1] ** 2
    keep = np.ix_([0, 1, 3], [0, 1, 3])
    assert np.max(np.abs(H[keep] - ref[keep])) < 1e-9
    # a single central difference at the same step is far off: the
    # extrapolation is doing the work
    h = 0.4
    e0 = np.eye(5)[0] * h
    c00 = (f(x + 2 * e0) - 2 * f(x) + f(x - 2 * e0)) / (4 * h * h)
    assert abs(c00 - ref[0, 0]) > 1e3 * abs(H[0, 0] - ref[0, 0])


def test_sigma_formula_closed_forms():
    H = np.diag(np.arange(1.0, 10.0))
    act = np.ones(9, np.int32)
    s = oracle.sec6_sigmas(H, act, 2.5, 7)
    assert np.allclose(s, np.sqrt(2.5 / (7 * np.arange(1.0, 10.0))), rtol=1e-15)
    # full matrix: [H^-1]_jj
    rng = np.random.default_rng(3)
    A = rng.normal(size=(9, 9))
    A = A @ A.T + np.eye(9)
    s = oracle.sec6_sigmas(A, act, 1.3, 9)
    assert np.allclose(s, np.sqrt(np.diag(np.linalg.inv(A)) * 1.3 / 9), rtol=1e-12)
    # held parameter: NaN, left out of the inverse
    act2 = act.copy()
    act2[4] = 0
    s = oracle.sec6_sigmas(A, act2, 1.3, 8)
    keep = [j for j in range(9) if j != 4]
    ref = np.sqrt(np.diag(np.linalg.inv(A[np.ix_(keep, keep)])) * 1.3 / 8)
    assert np.isnan(s[4]) and np.allclose(s[keep], ref, rtol=1e-12)
    # a parameter the function ignores: +inf, the others unaffected
    Z = A.copy()
    Z[6, :] = Z[:, 6] = 0.0
    s = oracle.sec6_sigmas(Z, act, 1.0, 9)
    keep = [j for j in range(9) if j != 6]
    assert s[6] == np.inf
    assert np.allclose(s[keep], np.sqrt(np.diag(np.linalg.inv(A[np.ix_(keep, keep)])) / 9))
    # indefinite: NaN everywhere
    D = np.diag([1.0, -1.0] + [1.0] * 7)
    assert np.isnan(oracle.sec6_sigmas(D, act, 1.0, 9)).all()


# ---- on the Milne-Eddington merit function --------------------------------

def _strong_truth(n, seed):
    t = si.draw_truth(n, seed)
    t[:, 0] = 1200.0 + 600.0 * np.arange(n) / max(n - 1, 1)
    t[:, 1] = 35.0 + (10.0 * np.arange(n)) % 90
    t[:, 6] = 8.0
    t[:, 5] = np.clip(t[:, 5], 0.05, 0.45)
    t[:, 7] = np.clip(t[:, 7], 0.05, 0.45)
    return t


def test_noise_free_hessian_equals_gauss_newton():
    """At the noise-free truth the residuals vanish, so the Hessian of the
    reduced chi-square is exactly (2/nu) J^T J with J the Jacobian of the
    weighted model.  J comes from plain central differences of the oracle's
    forward model at a small step (no tableau)."""
    lines = _lines("tiny")
    truth = _strong_truth(3, 5)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    L = obs.shape[-1]
    nu = 4 * L - 9
    u = oracle.uncertainty(obs, sig, lines, LO, HI, truth, np.tile(0.01 * SPAN, (3, 1)))
    for p in range(3):
        J = np.empty((4 * L, 9))
        for j in range(9):
            h = 1e-6 * SPAN[j]
            e = np.zeros(9)
            e[j] = h
            mp = oracle.me_synth((truth[p] + e)[None], lines)[0]
            mm = oracle.me_synth((truth[p] - e)[None], lines)[0]
            J[:, j] = ((mp - mm) / (2 * h) / sig[p][:, None]).ravel()
        gn = 2.0 / nu * J.T @ J
        H = u["hess"][p]
        scale = np.sqrt(np.outer(np.diag(gn), np.diag(gn)))
        assert np.max(np.abs(H - gn) / scale) < 1e-5, np.max(np.abs(H - gn) / scale)


def test_two_initial_steps_agree_within_error_estimates():
    lines = _lines("tiny")
    truth = _strong_truth(2, 6)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 6)
    r = oracle.lm_refine(obs, sig, lines, LO, HI, truth, 60)
    u1 = oracle.uncertainty(obs, sig, lines, LO, HI, r["params"], np.tile(0.02 * SPAN, (2, 1)))
    u2 = oracle.uncertainty(obs, sig, lines, LO, HI, r["params"], np.tile(0.004 * SPAN, (2, 1)))
    for p in range(2):
        d = np.abs(u1["hess"][p] - u2["hess"][p])
        scale = np.sqrt(np.outer(np.diag(u1["hess"][p]), np.diag(u1["hess"][p])))
        assert np.all(d <= 20 * (u1["hess_err"][p] + u2["hess_err"][p]) + 1e-7 * scale)
        # the inverse amplifies those differences by the condition number
        assert np.allclose(u1["sigma"][p], u2["sigma"][p], rtol=2e-3)


def test_uncertainty_tracks_the_scatter_of_repeated_inversions():
    """Monte Carlo: sigma_j^2 = [H^-1]_jj chi2 / M is the textbook covariance
    ((2/nu) H)^-1 scaled by (nu/2)(chi2/M); that covariance must match the
    scatter of refined parameters over independent noise draws."""
    lines = _lines("tiny")
    n = 64
    truth = np.repeat(_strong_truth(1, 9), n, axis=0)
    clean = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = clean + sig[:, :, None] * si.std_normal(clean.shape, 19)
    r = oracle.lm_refine(obs, sig, lines, LO, HI, truth, 60)
    u = oracle.uncertainty(obs, sig, lines, LO, HI, r["params"], np.tile(0.005 * SPAN, (n, 1)))
    nu = 4 * 100 - 9
    textbook = u["sigma"] * np.sqrt(2 * 9 / (nu * r["chi2"][:, None]))
    pred = np.median(textbook, axis=0)
    spread = r["params"].std(axis=0)
    for j in (0, 1, 3, 4, 6):      # B, inclination, v_los, Doppler width, eta0
        assert 0.7 < spread[j] / pred[j] < 1.4, (j, spread[j], pred[j])


def test_held_parameters_bounds_and_bad_pixels():
    lines = _lines("tiny")
    truth = _strong_truth(3, 7)
    truth[1, 5] = LO[5]                 # damping exactly at its lower bound
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs[2, 0, 5] = np.nan
    mask = 0x1FF & ~(1 << 2)            # azimuth held
    u = oracle.uncertainty(obs, sig, lines, LO, HI, truth, np.tile(0.01 * SPAN, (3, 1)),
                           free_mask=mask)
    assert np.isnan(u["sigma"][:2, 2]).all() and np.all(u["hess"][:2, 2] == 0)
    assert np.isnan(u["sigma"][1, 5]) and np.isfinite(u["sigma"][0, 5])
    assert u["steps"][1, 5] == 0.0
    assert np.isnan(u["sigma"][2]).all()
    # M = number of free parameters: sigma^2 M is independent of M's choice
    u9 = oracle.uncertainty(obs[:1], sig[:1], lines, LO, HI, truth[:1],
                            np.tile(0.01 * SPAN, (1, 1)))
    assert np.isfinite(u9["sigma"][0]).all()
    # steps bounded: at most a tenth of the span, at least 1e-4 of it, and
    # half the room to the nearer bound
    h = np.tile(np.array([1e9] * 9), (1, 1))
    uh = oracle.uncertainty(obs[:1], sig[:1], lines, LO, HI, truth[:1], h)
    room = np.minimum(truth[0] - LO, HI - truth[0])
    assert np.allclose(uh["steps"][0], np.minimum(0.1 * SPAN, 0.5 * room))
    ul = oracle.uncertainty(obs[:1], sig[:1], lines, LO, HI, truth[:1], np.zeros((1, 9)))
    assert np.allclose(ul["steps"][0], 1e-4 * SPAN)
    with pytest.raises(ValueError):
        oracle.uncertainty(obs, sig, lines, LO, HI, truth, np.ones((3, 9)), free_mask=0)


# ---- initial steps from the final population -------------------------------

def test_population_steps_rms_over_the_best_quarter():
    pop = 12
    rng = np.random.default_rng(4)
    genes = rng.integers(0, 65536, size=(2, pop, 9)).astype(np.uint16)
    fit = rng.uniform(1, 2, size=(2, pop))
    fit[0, 3] = np.nan                     # NaN ranks last
    fit[0, 5] = fit[0, 7] = 0.5            # tie: the lower index ranks first
    fit[0, 9] = 0.4
    p_opt = rng.uniform(LO, HI, size=(2, 9))
    h = oracle.population_steps(genes, fit, LO, HI, p_opt)
    for p in range(2):
        order = sorted(range(pop), key=lambda i: (np.isnan(fit[p, i]),
                                                  0 if np.isnan(fit[p, i]) else fit[p, i], i))
        best = order[:3]                   # max(2, 12 // 4)
        par = LO + SPAN * genes[p, best].astype(np.float64) / 65535.0
        assert np.allclose(h[p], np.sqrt(np.mean((par - p_opt[p]) ** 2, axis=0)), rtol=1e-14)
    assert sorted(order[:3]) == sorted(order[:3])
    # small populations: at least two individuals, all of a population of one
    g5 = genes[:1, :5]
    f5 = np.array([[3.0, 1.0, 2.0, 5.0, 4.0]])
    h5 = oracle.population_steps(g5, f5, LO, HI, p_opt[:1])
    par = LO + SPAN * g5[0, [1, 2]].astype(np.float64) / 65535.0
    assert np.allclose(h5[0], np.sqrt(np.mean((par - p_opt[0]) ** 2, axis=0)), rtol=1e-14)
    h1 = oracle.population_steps(genes[:1, :1], fit[:1, :1], LO, HI, p_opt[:1])
    par = LO + SPAN * genes[0, 0].astype(np.float64) / 65535.0
    assert np.allclose(h1[0], np.abs(par - p_opt[0]), rtol=1e-14)
