"""Pins of the oracle's non-magnetic pre-fit (Sec. 5.3), of its per-pixel
search boxes (Sec. 5.3 ranges, Sec. 5.5 polarity) and of the genetic
algorithm run inside per-pixel boxes.

The pre-fit is pinned by what the mathematics fixes: on a noise-free
non-magnetic observation the model is exact, so the fit must return the truth;
the held parameters come back untouched; with no free parameter the fit is the
identity; the Q, U and V observations cannot steer it (the model's Q, U and V
vanish at B = 0).  The polarity rule is pinned by the weak-field relation
V ~ -cos(incl) dI/dlambda, on forward-model profiles of known inclination, and
by its antisymmetry in V.  Per-pixel boxes are pinned by reduction to the
common-box algorithm: a pixel run in its own box equals that pixel run alone
with its box as the common one."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle import firstguess as ofg
from oracle import searchbox as osb

LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _lines(kind):
    out = []
    for line, n in si.line_set(kind):
        st, sp = si.grid(line, n)
        out.append(oracle.make_line(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"],
                                    st, sp, n))
    return out


def _nonmagnetic(n, seed):
    t = si.draw_truth(n, seed)
    t[:, 0] = 0.0
    return t


def test_prefit_recovers_a_nonmagnetic_truth():
    lines = _lines("slit")
    truth = _nonmagnetic(6, 3)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    rng = np.random.default_rng(4)
    start = np.clip(truth + (HI - LO) * rng.normal(0, 0.02, truth.shape), LO, HI)
    r = oracle.prefit(obs, sig, lines, LO, HI, start, 60)
    free = [3, 4, 5, 6, 7, 8]
    err = np.abs(r["params"][:, free] - truth[:, free]) / (HI - LO)[free]
    assert err.max() < 1e-5, err.max()
    assert np.all(r["chi2"] < 1e-8)
    # B is held at 0 and the angles keep their starting values (up to the
    # rounding of the trip through normalised coordinates)
    assert np.all(r["params"][:, 0] == 0.0)
    assert np.allclose(r["params"][:, 1:3], start[:, 1:3], rtol=0, atol=1e-12 * 180.0)


def test_fit_with_nothing_free_is_the_identity():
    lines = _lines("tiny")
    truth = si.draw_truth(4, 5)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    start = si.draw_truth(4, 6)
    r = oracle.lm_refine(obs, sig, lines, LO, HI, start, 10, free_mask=0)
    assert np.allclose(r["params"], start, rtol=0, atol=1e-12 * np.max(HI - LO))
    assert np.all(r["iters"] == 0)
    c = oracle.chi2(start[:, None], obs, sig, lines)[:, 0]
    assert np.allclose(r["chi2"], c, rtol=1e-12)


def test_prefit_ignores_the_polarisation_profiles():
    lines = _lines("slit")
    truth = si.draw_truth(5, 7)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 7)
    start = ofg.first_guess(obs, lines, LO, HI)
    a = oracle.prefit(obs, sig, lines, LO, HI, start, 30)
    o2 = obs.copy()
    o2[:, 1:] = 0.0
    b = oracle.prefit(o2, sig, lines, LO, HI, start, 30)
    assert np.allclose(a["params"], b["params"], rtol=0, atol=1e-6 * np.max(HI - LO))


def test_prefit_needs_a_box_with_zero_field():
    lo = LO.copy()
    lo[0] = 10.0
    with pytest.raises(ValueError):
        oracle.prefit(np.zeros((1, 4, 8)), np.ones((1, 4)), _lines("tiny"), lo, HI,
                      np.zeros((1, 9)), 1)


def _magnetic(incl, n=8, seed=9):
    t = si.draw_truth(n, seed)
    t[:, 0] = 1500.0
    t[:, 1] = incl
    return t


@pytest.mark.parametrize("incl,expect", [(25.0, (0.0, 90.0)), (155.0, (90.0, 180.0))])
def test_polarity_follows_the_lobe_order(incl, expect):
    lines = _lines("slit")
    truth = _magnetic(incl)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 10)
    box = osb.search_box(obs, sig, lines, LO, HI, n_sigma=3.0)
    assert np.all(box[:, 0, 1] == expect[0]) and np.all(box[:, 1, 1] == expect[1])
    # every other range is the common one
    others = [j for j in range(9) if j != 1]
    assert np.array_equal(box[:, 0, others], np.broadcast_to(LO[others], (8, 8)))
    assert np.array_equal(box[:, 1, others], np.broadcast_to(HI[others], (8, 8)))
    # V -> -V flips the decision; no Stokes V leaves the range open
    flip = obs.copy()
    flip[:, 3] *= -1
    fb = osb.search_box(flip, sig, lines, LO, HI, n_sigma=3.0)
    assert np.all(fb[:, 0, 1] == (90.0 if expect[0] == 0.0 else 0.0))
    none = obs.copy()
    none[:, 3] = 0.0
    nb = osb.search_box(none, sig, lines, LO, HI, n_sigma=3.0)
    assert np.all(nb[:, 0, 1] == LO[1]) and np.all(nb[:, 1, 1] == HI[1])


def test_polarity_off_and_prefit_off_give_the_common_box():
    lines = _lines("tiny")
    truth = _magnetic(40.0, 3)
    obs = oracle.me_synth(truth, lines)
    box = osb.search_box(obs, si.sigma_for(truth), lines, LO, HI, prefit=None, n_sigma=0.0)
    assert np.array_equal(box[:, 0], np.broadcast_to(LO, (3, 9)))
    assert np.array_equal(box[:, 1], np.broadcast_to(HI, (3, 9)))


def test_prefit_ranges_lie_in_the_common_box_and_hold_the_prefit():
    lines = _lines("slit")
    truth = si.draw_truth(40, 11)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 11)
    pf = oracle.prefit(obs, sig, lines, LO, HI, ofg.first_guess(obs, lines, LO, HI), 20)["params"]
    box = osb.search_box(obs, sig, lines, LO, HI, prefit=pf, n_sigma=0.0)
    assert np.all(box[:, 0] >= LO) and np.all(box[:, 1] <= HI) and np.all(box[:, 1] >= box[:, 0])
    # the pre-fit value itself is always inside its ranges (the windows open
    # upwards of it for the Doppler width and damping, around it otherwise)
    for j in (4, 5, 6, 8):
        assert np.all((box[:, 0, j] <= pf[:, j]) & (pf[:, j] <= box[:, 1, j])), j
    # the Doppler width and damping keep their lower bound; untouched ranges stay
    assert np.all(box[:, 0, [4, 5]] == LO[[4, 5]])
    for j in (0, 1, 2, 3, 7):
        assert np.all(box[:, 0, j] == LO[j]) and np.all(box[:, 1, j] == HI[j])


def _ga_problem(n, seed):
    lines = _lines("tiny")
    truth = si.draw_truth(n, seed)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return lines, obs, sig


def _boxes(n, seed):
    rng = np.random.default_rng(seed)
    a = LO + (HI - LO) * rng.uniform(0, 0.5, (n, 9))
    b = a + (HI - LO) * rng.uniform(0.2, 0.5, (n, 9))
    return np.stack([a, np.minimum(b, HI)], axis=1)


def test_pixel_boxes_reduce_to_single_pixel_runs():
    lines, obs, sig = _ga_problem(4, 12)
    box = _boxes(4, 13)
    kw = dict(pop=16, generations=5, k=4, p_cross=0.85, p_mut=0.05, seed=3, want_population=True)
    res = oracle.ga_invert(obs, sig, lines, LO, HI, pixel_box=box, **kw)
    for p in range(4):
        alone = oracle.ga_invert(obs[p:p + 1], sig[p:p + 1], lines, box[p, 0], box[p, 1],
                                 pixel_base=p, **kw)
        assert np.array_equal(res["genes"][p], alone["genes"][0])
        assert np.array_equal(res["params"][p], alone["params"][0])
        # every individual decodes inside its pixel's box
        par = oracle.decode(res["genes"][p], box[p, 0], box[p, 1])
        assert np.all(par >= box[p, 0]) and np.all(par <= box[p, 1])
    # the common box given per pixel changes nothing
    same = oracle.ga_invert(obs, sig, lines, LO, HI, pixel_box=np.stack([np.broadcast_to(LO, (4, 9)),
                                                                         np.broadcast_to(HI, (4, 9))], 1), **kw)
    plain = oracle.ga_invert(obs, sig, lines, LO, HI, **kw)
    assert np.array_equal(same["genes"], plain["genes"])


def test_invalid_pixel_box_gives_status_3():
    lines, obs, sig = _ga_problem(3, 14)
    box = _boxes(3, 15)
    box[1, 1, 4] = box[1, 0, 4] - 1e-3       # hi < lo
    box[2, 0, 0] = np.nan
    res = oracle.ga_invert(obs, sig, lines, LO, HI, pop=8, generations=2, k=2, p_cross=0.8,
                           p_mut=0.05, seed=1, pixel_box=box)
    assert list(res["status"]) == [0, 3, 3]
    assert np.all(np.isnan(res["params"][1:])) and np.isfinite(res["params"][0]).all()
