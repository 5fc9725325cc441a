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


# ---- the four separate seeds of Sec. 5.5 -----------------------------------

WF, IR, COG, NM = range(4)


def test_seeds_in_the_weak_field_limit():
    """At 30 G the weak-field relations hold to first order: both field
    seeds recover the longitudinal field of a longitudinal field to 2 %
    (the integral relation exactly so: sum |V| = C gbar |B_par| sum |I'|
    when V is proportional to I'), the centre-of-gravity seed too."""
    lines = _lines()
    P = np.array([_model(B=30.0, incl=0.0), _model(B=30.0, incl=180.0)])
    S = fg.seeds(oracle.me_synth(P, lines), lines, LO, HI)
    for k in (WF, IR, COG):
        assert abs(S[0, k, 0] - 30.0) < 0.02 * 30.0, k
        assert S[0, k, 1] < 2.0 and S[1, k, 1] > 178.0, k
    assert abs(S[0, COG, 0] - fg.first_guess(oracle.me_synth(P, lines), lines, LO, HI)[0, 0]) \
        < 1e-9


@pytest.mark.parametrize("chi", [20.0, 75.0, 140.0])
def test_transverse_seeds_recover_the_azimuth(chi):
    lines = _lines()
    S = fg.seeds(oracle.me_synth(_model(B=300.0, incl=90.0, azim=chi)[None], lines), lines,
                 LO, HI)[0]
    for k in (WF, IR):
        d = abs(S[k, 2] - chi) % 180.0
        assert min(d, 180.0 - d) < 1.0, k
        assert abs(S[k, 1] - 90.0) < 2.0, k
    # the integral azimuth also holds for a strong field (no weak-field shape)
    S = fg.seeds(oracle.me_synth(_model(B=2000.0, incl=60.0, azim=chi)[None], lines), lines,
                 LO, HI)[0]
    d = abs(S[IR, 2] - chi) % 180.0
    assert min(d, 180.0 - d) < 3.0


def test_seeds_invert_profiles_that_obey_the_weak_field_relations_exactly():
    """Profiles built to satisfy V = -C gbar B_par I' and (Q, U) = -(1/4) C^2
    gbar^2 B_perp^2 (cos 2chi, sin 2chi) I'' at every sample (I from the
    oracle's non-magnetic model, derivatives by the same differences the
    seeds use): the weak-field seed's least squares and the integral
    relations both return B_par, B_perp and chi to rounding."""
    lines = _lines()
    for bpar, bperp, chi in ((120.0, 300.0, 35.0), (-80.0, 500.0, 160.0), (400.0, 50.0, 95.0)):
        obs = oracle.me_synth(_model()[None], lines)
        off = 0
        for ln in lines:
            n = ln.nlam
            I = obs[0, 0, off:off + n]
            d1, d2 = fg._derivs(I, ln.step)
            C = fg.ZEEMAN * ln.lambda0 ** 2
            g = fg.gbar_of(ln)
            obs[0, 3, off:off + n] = -C * g * bpar * d1
            lin = -0.25 * (C * g) ** 2 * bperp ** 2 * d2
            obs[0, 1, off:off + n] = lin * np.cos(np.radians(2 * chi))
            obs[0, 2, off:off + n] = lin * np.sin(np.radians(2 * chi))
            off += n
        S = fg.seeds(obs, lines, np.array([0.0, 0, 0, -7.5, 0.02, 0, 1, 0, 0.5]),
                     np.array([3000.0, 180, 180, 7.5, 0.05, 0.5, 30, 0.5, 1.0]))[0]
        B = np.hypot(bpar, bperp)
        inc = np.degrees(np.arctan2(bperp, bpar))
        for k in (WF, IR):
            assert np.allclose(S[k, :3], [B, inc, chi], rtol=1e-9, atol=1e-7), (k, S[k, :3])


def test_seed_layout_unseeded_angles_and_shared_thermodynamics():
    lines = _lines()
    truth = si.draw_truth(20, 8)
    obs = oracle.me_synth(truth, lines)
    S = fg.seeds(obs, lines, LO, HI)
    g = fg.first_guess(obs, lines, LO, HI)
    assert S.shape == (20, 4, 9)
    assert np.all(S[:, NM, 0] == 0.0) and np.isnan(S[:, NM, 1:3]).all()
    assert np.isnan(S[:, COG, 2]).all() and np.isin(S[:, COG, 1], (0.0, 180.0)).all()
    for k in range(4):
        assert np.array_equal(S[:, k, 3:], g[:, 3:])
    fin = ~np.isnan(S)
    lo = np.broadcast_to(LO, S.shape)
    hi = np.broadcast_to(HI, S.shape)
    assert np.all(S[fin] >= lo[fin]) and np.all(S[fin] <= hi[fin])


def test_seeds_follow_the_polarity_box_and_symmetries():
    lines = _lines()
    P = np.array([_model(B=400.0, incl=40.0, azim=70.0), _model(B=900.0, incl=130.0, azim=10.0)])
    obs = oracle.me_synth(P, lines)
    S = fg.seeds(obs, lines, LO, HI)
    # V -> -V mirrors every seeded inclination
    flip = obs.copy()
    flip[:, 3] *= -1
    Sf = fg.seeds(flip, lines, LO, HI)
    for k in (WF, IR, COG):
        assert np.allclose(Sf[:, k, 1], 180.0 - S[:, k, 1], atol=1e-9), k
        assert np.allclose(Sf[:, k, 0], S[:, k, 0], rtol=1e-9), k
    # a rotation of Q, U by 2 theta turns the seeded azimuths by theta
    th = np.radians(33.0)
    rot = obs.copy()
    rot[:, 1] = np.cos(2 * th) * obs[:, 1] - np.sin(2 * th) * obs[:, 2]
    rot[:, 2] = np.sin(2 * th) * obs[:, 1] + np.cos(2 * th) * obs[:, 2]
    Sr = fg.seeds(rot, lines, LO, HI)
    for k in (WF, IR):
        d = (Sr[:, k, 2] - S[:, k, 2] - 33.0) % 180.0
        assert np.all(np.minimum(d, 180.0 - d) < 1e-6), k
    # a polarity box on the other side reflects the inclination into it
    box = np.stack([np.tile(LO, (2, 1)), np.tile(HI, (2, 1))], axis=1)
    box[0, 0, 1], box[0, 1, 1] = 90.0, 180.0
    box[1, 0, 1], box[1, 1, 1] = 0.0, 90.0
    box[0, 1, 0] = 200.0                  # and B capped
    Sb = fg.seeds(obs, lines, LO, HI, box=box)
    for k in (WF, IR, COG):
        assert np.isclose(Sb[0, k, 1], 180.0 - S[0, k, 1]) and 90.0 <= Sb[0, k, 1] <= 180.0
        assert np.isclose(Sb[1, k, 1], 180.0 - S[1, k, 1]) and Sb[1, k, 1] <= 90.0
        assert Sb[0, k, 0] <= 200.0
