"""Pins of the oracle's heuristic first guesses (Sec. 5.5 seeds): what the
centre-of-gravity and weak-field relations fix for the oracle's own exact
synthesis -- the line-of-sight velocity of a non-magnetic line, the
longitudinal field of a weak field (the centre-of-gravity separation of I+V
and I-V is exactly 2 C gbar B cos(incl) there), the azimuth of a weak
transverse field, and the symmetries (V -> -V mirrors the inclination, a
rotation of Q and U by 2 theta turns the azimuth by theta)."""
import numpy as np
import pytest

import oracle
from oracle import firstguess as fg
import synth_inputs as si

LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _lines(kind="slit"):
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set(kind)]


def _model(B=0.0, incl=0.0, azim=0.0, vlos=0.0, dop=0.03, damp=0.1, eta0=5.0, S0=0.25, S1=0.75):
    return np.array([B, incl, azim, vlos, dop, damp, eta0, S0, S1])


def test_gbar_is_the_effective_lande_factor():
    lines = _lines()
    assert abs(fg.gbar_of(lines[0]) - 5.0 / 3.0) < 1e-12     # Table 1: 1.667
    assert abs(fg.gbar_of(lines[1]) - 2.5) < 1e-12            # Table 1: 2.500


@pytest.mark.parametrize("v", [-2.0, 0.0, 3.0])
def test_velocity_of_a_non_magnetic_line(v):
    lines = _lines()
    g = fg.first_guess(oracle.me_synth(_model(vlos=v)[None], lines), lines, LO, HI)[0]
    assert abs(g[3] - v) < 0.02
    assert g[0] < 1.0


def test_weak_longitudinal_field():
    lines = _lines()
    P = np.array([_model(B=150.0, incl=0.0), _model(B=150.0, incl=180.0),
                  _model(B=80.0, incl=0.0, vlos=1.5)])
    g = fg.first_guess(oracle.me_synth(P, lines), lines, LO, HI)
    assert abs(g[0, 0] - 150.0) < 0.02 * 150.0 and g[0, 1] < 1.0
    assert abs(g[1, 0] - 150.0) < 0.02 * 150.0 and g[1, 1] > 179.0
    assert abs(g[2, 0] - 80.0) < 0.02 * 80.0 and abs(g[2, 3] - 1.5) < 0.02


@pytest.mark.parametrize("chi", [30.0, 120.0, 170.0])
def test_weak_transverse_field_azimuth(chi):
    lines = _lines()
    g = fg.first_guess(oracle.me_synth(_model(B=500.0, incl=90.0, azim=chi)[None], lines),
                       lines, LO, HI)[0]
    d = abs(g[2] - chi) % 180.0
    assert min(d, 180.0 - d) < 1.0
    assert abs(g[1] - 90.0) < 1.0


def test_symmetries():
    lines = _lines()
    rng = np.random.default_rng(2)
    P = np.array([_model(B=b, incl=i, azim=a) for b, i, a in
                  zip(rng.uniform(200, 1500, 6), rng.uniform(10, 170, 6), rng.uniform(0, 180, 6))])
    obs = oracle.me_synth(P, lines)
    g = fg.first_guess(obs, lines, LO, HI)
    flip = obs.copy()
    flip[:, 3] *= -1
    gf = fg.first_guess(flip, lines, LO, HI)
    assert np.allclose(gf[:, 0], g[:, 0], rtol=1e-9)
    assert np.allclose(gf[:, 1], 180.0 - g[:, 1], atol=1e-9)
    th = np.radians(25.0)
    rot = obs.copy()
    rot[:, 1] = np.cos(2 * th) * obs[:, 1] - np.sin(2 * th) * obs[:, 2]
    rot[:, 2] = np.sin(2 * th) * obs[:, 1] + np.cos(2 * th) * obs[:, 2]
    gr = fg.first_guess(rot, lines, LO, HI)
    d = (gr[:, 2] - g[:, 2] - 25.0) % 180.0
    assert np.all(np.minimum(d, 180.0 - d) < 1e-6)


def test_guesses_stay_in_the_box():
    lines = _lines()
    truth = si.draw_truth(200, 4)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 4)
    g = fg.first_guess(obs, lines, LO, HI)
    assert np.all(g >= LO) and np.all(g <= HI) and np.isfinite(g).all()
    # informative where the approximations hold: velocity and field strength
    assert np.median(np.abs(g[:, 3] - truth[:, 3])) < 0.1
    assert np.median(np.abs(g[:, 0] - truth[:, 0])) < 0.75 * np.median(np.abs(truth[:, 0] - 1500))
