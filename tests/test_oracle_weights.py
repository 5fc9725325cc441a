"""Pins of the oracle's inverse-max weights (Sec. 5.4): a worked example by
hand, what zero field and the Zeeman symmetries fix, and the properties the
scheme exists for (every weighted Q, U, V profile peaks at exactly 1 in
magnitude; the weighted I depression spans exactly 1)."""
import numpy as np

import oracle
from oracle import weights as ow
import synth_inputs as si


def _lines():
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set("slit")]


def test_worked_example():
    # I: continuum 1.0, core 0.4; Q peaks at |-0.3|; U at 0.05; V is zero.
    obs = np.array([[[1.0, 0.4, 0.7, 0.95],
                     [0.0, -0.3, 0.2, 0.0],
                     [0.05, 0.0, -0.01, 0.02],
                     [0.0, 0.0, 0.0, 0.0]]])
    s = ow.invmax_sigma(obs, floor=1e-3)
    assert np.array_equal(s, [[0.6, 0.3, 0.05, 1e-3]])


def test_zero_field_gives_the_floor_for_polarisation():
    truth = si.draw_truth(5, seed=4)
    truth[:, 0] = 0.0
    obs = oracle.me_synth(truth, _lines())
    s = ow.invmax_sigma(obs, floor=2e-3)
    assert np.all(s[:, 1:] == 2e-3)
    # the I depression: largest minus smallest I of the pixel
    assert np.allclose(s[:, 0], obs[:, 0].max(axis=1) - obs[:, 0].min(axis=1), rtol=0, atol=0)
    assert np.all(s[:, 0] > 0.05)


def test_weighted_profiles_peak_at_one():
    truth = si.draw_truth(40, seed=5)
    truth[:, 0] = np.linspace(200.0, 3000.0, 40)
    truth[:, 1] = np.clip(truth[:, 1], 20.0, 160.0)
    obs = oracle.me_synth(truth, _lines())
    s = ow.invmax_sigma(obs, floor=1e-9)
    for k in (1, 2, 3):
        assert np.allclose(np.max(np.abs(obs[:, k]), axis=1) / s[:, k], 1.0, rtol=1e-15, atol=0)
    span = (obs[:, 0].max(axis=1) - obs[:, 0].min(axis=1)) / s[:, 0]
    assert np.allclose(span, 1.0, rtol=1e-15, atol=0)


def test_symmetries():
    """Inclination 180 - incl turns V into -V and keeps I (the
    magneto-optical effects change Q and U), so the weights of I and V stay;
    an azimuth turned by 45 deg swaps the roles of Q and U; a scale c of the
    Stokes vector scales every sigma by c."""
    lines = _lines()
    t = si.draw_truth(6, seed=6)
    t[:, 0] = 1500.0
    obs = oracle.me_synth(t, lines)
    t2 = t.copy()
    t2[:, 1] = 180.0 - t[:, 1]
    obs2 = oracle.me_synth(t2, lines)
    s, s2 = ow.invmax_sigma(obs, 1e-9), ow.invmax_sigma(obs2, 1e-9)
    assert np.allclose(s2[:, [0, 3]], s[:, [0, 3]], rtol=1e-12)
    # azimuth + 45 deg turns Q into U (and U into -Q)
    t3 = t.copy()
    t3[:, 2] = (t[:, 2] + 45.0) % 180.0
    s3 = ow.invmax_sigma(oracle.me_synth(t3, lines), 1e-9)
    assert np.allclose(s3[:, 1], s[:, 2], rtol=1e-9)
    assert np.allclose(s3[:, 2], s[:, 1], rtol=1e-9)
    assert np.allclose(ow.invmax_sigma(3.0 * obs, 1e-9), 3.0 * s, rtol=1e-15)


def test_non_finite_pixel():
    obs = np.ones((2, 4, 8))
    obs[1, 2, 3] = np.nan
    s = ow.invmax_sigma(obs, 1e-3)
    assert np.all(np.isnan(s[1])) and np.all(np.isfinite(s[0]))
