"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
independent library routines (mpmath, scipy, sympy), brute-force quadrature,
published values (Table 1, Philox known answers) and physical invariants of the
Milne-Eddington solution (Sec. 5).
"""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

import oracle
import synth_inputs as si
from conftest import read_table

SQPI = math.sqrt(math.pi)


# --------------------------------------------------------------------------- #
# Faddeeva / Voigt / Faraday-Voigt (Sec. 5)

def _w_mpmath(x, y):
    z = mpmath.mpc(x, y)
    return complex(mpmath.exp(-z * z) * mpmath.erfc(-1j * z))


def test_faddeeva_vs_mpmath():
    mpmath.mp.dps = 30
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-45, 45, 150), rng.uniform(-6, 6, 150), [0.0, 3.7, -5.2]])
    ys = np.concatenate([rng.uniform(0, 0.6, 300), [0.0, 0.0, 1.4]])
    ys[::7] = 0.0
    ys[1::11] = 1e-4
    got = oracle.faddeeva(xs, ys)
    ref = np.array([_w_mpmath(x, y) for x, y in zip(xs, ys)])
    assert np.max(np.abs(got - ref)) < 2e-15


def test_faddeeva_vs_scipy_grid():
    x = np.linspace(-50, 50, 1001)
    for y in (0.0, 1e-3, 0.05, 0.5, 1.5):
        assert np.max(np.abs(oracle.faddeeva(x, y) - special.wofz(x + 1j * y))) < 5e-15


@pytest.mark.parametrize("a", [0.02, 0.3, 0.5])
@pytest.mark.parametrize("v", [0.0, 0.7, 2.5, 6.0, 15.0])
def test_voigt_faraday_vs_quadrature(a, v):
    # H = (a/pi) int exp(-y^2)/((v-y)^2+a^2) dy ; L = (1/pi) int (v-y) exp(-y^2)/((v-y)^2+a^2) dy
    fH = lambda y: math.exp(-y * y) / ((v - y) ** 2 + a * a)
    fL = lambda y: (v - y) * math.exp(-y * y) / ((v - y) ** 2 + a * a)
    pts = sorted({v, 0.0})
    H = a / math.pi * sum(integrate.quad(fH, lo, hi, points=[p for p in pts if lo < p < hi],
                                         limit=400, epsabs=1e-14, epsrel=1e-12)[0]
                          for lo, hi in ((-40, 40),))
    L = 1 / math.pi * integrate.quad(fL, -40, 40, points=pts, limit=400, epsabs=1e-14,
                                     epsrel=1e-12)[0]
    w = oracle.faddeeva(v, a)
    assert abs(w.real - H) < 1e-10
    assert abs(w.imag - L) < 1e-10


def test_voigt_closed_forms():
    v = np.linspace(-30, 30, 601)
    w0 = oracle.faddeeva(v, 0.0)
    # H(0, v) = exp(-v^2); L(0, v) = (2/sqrt(pi)) Dawson(v)
    assert np.max(np.abs(w0.real - np.exp(-v * v))) < 1e-15
    assert np.max(np.abs(w0.imag - 2 / SQPI * special.dawsn(v))) < 2e-15
    # H(a, 0) = erfcx(a), L(a, 0) = 0
    a = np.linspace(0, 1.5, 31)
    wa = oracle.faddeeva(0.0, a)
    assert np.max(np.abs(wa.real - special.erfcx(a))) < 1e-14
    assert np.max(np.abs(wa.imag)) < 1e-14


def test_voigt_normalisation_and_asymptote():
    a = 0.05
    v = np.linspace(-400, 400, 160001)
    H = oracle.faddeeva(v, a).real
    tail = 2 * a / (SQPI * 400.0)           # analytic tail of a/(sqrt(pi) v^2) beyond |v| = 400
    assert abs(np.trapezoid(H, v) + tail - SQPI) < 2e-6
    for vv in (200.0, 1000.0):
        w = oracle.faddeeva(vv, a)
        assert abs(w.real / (a / (SQPI * vv * vv)) - 1) < 1e-4
        assert abs(w.imag / (1 / (SQPI * vv)) - 1) < 1e-4


# --------------------------------------------------------------------------- #
# Zeeman pattern (Sec. 5; Table 1)

def test_wigner3j_golden(golden_dir):
    for row in read_table(os.path.join(golden_dir, "wigner3j.txt")):
        j1, j2, j3, m1, m2, m3, val = map(float, row)
        assert abs(oracle.wigner3j(j1, j2, j3, m1, m2, m3) - val) < 1e-14


def test_wigner3j_vs_sympy():
    from sympy import Rational
    from sympy.physics.wigner import wigner_3j
    rng = np.random.default_rng(3)
    for _ in range(60):
        J1 = int(rng.integers(0, 9))
        J2 = 2
        J3 = int(rng.integers(0, 9))
        M1 = int(rng.integers(-J1, J1 + 1))
        M2 = int(rng.integers(-2, 3))
        M3 = -M1 - M2
        if (J1 + M1) % 2 or (J3 + M3) % 2 or (J1 + J2 + J3) % 2:
            continue
        ref = float(wigner_3j(Rational(J1, 2), Rational(J2, 2), Rational(J3, 2),
                              Rational(M1, 2), Rational(M2, 2), Rational(M3, 2)))
        assert abs(oracle.wigner3j(J1 / 2, J2 / 2, J3 / 2, M1 / 2, M2 / 2, M3 / 2) - ref) < 1e-14


def test_lande_factors_of_table1_terms():
    for line in (si.FE6301, si.FE6302):
        (Sl, Ll, Jl), (Su, Lu, Ju) = line["terms"]
        assert abs(oracle.lande_ls(Sl, Ll, Jl) - line["gl"]) < 1e-15
        assert abs(oracle.lande_ls(Su, Lu, Ju) - line["gu"]) < 1e-15


def test_zeeman_counts_sums_moments(golden_dir):
    table = {float(r[0]): float(r[3]) for r in read_table(os.path.join(golden_dir, "table1_lines.txt"))}
    for line, ncomp in ((si.FE6301, 12), (si.FE6302, 3)):
        q, s, st = oracle.zeeman(line["Jl"], line["gl"], line["Ju"], line["gu"])
        assert len(q) == ncomp
        for g in (-1, 0, 1):
            assert abs(st[q == g].sum() - 1.0) < 1e-14
        gbar = float(np.sum(st[q == 1] * s[q == 1]))
        assert abs(np.sum(st[q == -1] * s[q == -1]) + gbar) < 1e-14
        assert abs(np.sum(st[q == 0] * s[q == 0])) < 1e-14
        # effective Lande factor of Table 1
        assert abs(gbar - table[line["lambda0"]]) < 5e-4
        # closed-form effective Lande factor of the two levels
        gl, gu, Jl, Ju = line["gl"], line["gu"], line["Jl"], line["Ju"]
        geff = 0.5 * (gl + gu) + 0.25 * (gl - gu) * (Jl * (Jl + 1) - Ju * (Ju + 1))
        assert abs(gbar - geff) < 1e-14


def test_zeeman_normal_triplet():
    q, s, st = oracle.zeeman(1, 1.3, 1, 1.3)     # equal g: normal triplet with 6 components
    for g in (-1, 0, 1):
        assert np.allclose(s[q == g], g * 1.3)


# --------------------------------------------------------------------------- #
# Milne-Eddington synthesis invariants (Sec. 5)

def _lines(kind="slit", nlam=None):
    out = []
    for line, n in si.line_set(kind):
        n = nlam or n
        start, step = si.grid(line, n)
        out.append(oracle.make_line(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"],
                                    start, step, n))
    return out


def _params(n, seed=5):
    return si.draw_uniform_box(n, seed)


def test_zero_field_gives_no_polarisation():
    lines = _lines("slit", 64)
    p = _params(20)
    p[:, 0] = 0.0
    st = oracle.me_synth(p, lines)
    assert np.max(np.abs(st[:, 1:])) < 1e-15      # rounding of the group sums only
    # I = S0 + mu S1 / (1 + eta0 H) with the Doppler-shifted line centre
    off = 0
    for ln in lines:
        lam = ln.start + np.arange(ln.nlam) * ln.step
        for i in range(len(p)):
            lc = ln.lambda0 * (1 + p[i, 3] / 299792.458)
            H = special.wofz((lam - lc) / p[i, 4] + 1j * p[i, 5]).real
            ref = p[i, 7] + p[i, 8] / (1 + p[i, 6] * H)
            assert np.max(np.abs(st[i, 0, off:off + ln.nlam] - ref)) < 1e-13
        off += ln.nlam


def test_zero_opacity_gives_continuum():
    lines = _lines("slit", 32)
    p = _params(10)
    p[:, 6] = 0.0
    st = oracle.me_synth(p, lines)
    assert np.max(np.abs(st[:, 0] - (p[:, 7] + p[:, 8])[:, None])) < 1e-15
    assert np.max(np.abs(st[:, 1:])) < 1e-15


def _two_by_two_reference(line_kw, ln, par, mode):
    """Independent route for two special geometries, using scipy's Faddeeva
    and the component list: gamma = 0 decouples (I, V); gamma = 90, chi = 0
    decouples (I, Q)."""
    q, s, st = oracle.zeeman(line_kw["Jl"], line_kw["gl"], line_kw["Ju"], line_kw["gu"])
    lam = ln.start + np.arange(ln.nlam) * ln.step
    B, _, _, vlos, dop, a, eta0, S0, S1 = par
    lc = ln.lambda0 * (1 + vlos / 299792.458)
    dlb = 4.6686e-13 * ln.lambda0 ** 2 * B
    phi = {g: np.zeros(ln.nlam) for g in (-1, 0, 1)}
    for qq, ss, ww in zip(q, s, st):
        phi[qq] += ww * special.wofz((lam - lc - ss * dlb) / dop + 1j * a).real
    if mode == "long":
        k = 1 + eta0 * 0.5 * (phi[-1] + phi[1])
        etaV = 0.5 * eta0 * (phi[1] - phi[-1])
        den = k * k - etaV * etaV
        return S0 + S1 * k / den, -S1 * etaV / den
    k = 1 + 0.5 * eta0 * (phi[0] + 0.5 * (phi[-1] + phi[1]))
    etaQ = 0.5 * eta0 * (phi[0] - 0.5 * (phi[-1] + phi[1]))
    den = k * k - etaQ * etaQ
    return S0 + S1 * k / den, -S1 * etaQ / den


@pytest.mark.parametrize("mode", ["long", "trans"])
def test_special_geometries_independent_route(mode):
    lines = _lines("slit", 96)
    p = _params(8, seed=11)
    if mode == "long":
        p[:, 1] = 0.0
    else:
        p[:, 1] = 90.0
        p[:, 2] = 0.0
    st = oracle.me_synth(p, lines)
    off = 0
    for (kw, _), ln in zip(si.line_set("slit"), lines):
        for i in range(len(p)):
            I_ref, X_ref = _two_by_two_reference(kw, ln, p[i], mode)
            sl = slice(off, off + ln.nlam)
            assert np.max(np.abs(st[i, 0, sl] - I_ref)) < 1e-13
            if mode == "long":
                assert np.max(np.abs(st[i, 3, sl] - X_ref)) < 1e-13
                assert np.max(np.abs(st[i, 1:3, sl])) < 1e-15
            else:
                assert np.max(np.abs(st[i, 1, sl] - X_ref)) < 1e-13
                assert np.max(np.abs(st[i, 2:4, sl])) < 1e-15
        off += ln.nlam


def test_weak_field_limit():
    # V ~ -gbar dlambda_B cos(gamma) dI/dlambda + O(B^2)
    line = si.FE6302
    n = 4001
    start, step = si.grid(line, n)
    ln = oracle.make_line(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"],
                          start, step, n)
    base = np.array([0.0, 30.0, 20.0, 0.4, 0.03, 0.2, 8.0, 0.2, 0.8])
    errs = []
    for B in (10.0, 20.0, 40.0):
        p = base.copy()
        p[0] = B
        st = oracle.me_synth(p[None], [ln])[0]
        dI = np.gradient(st[0], step)
        dlb = 4.6686e-13 * line["lambda0"] ** 2 * B
        Vw = -2.5 * dlb * math.cos(math.radians(p[1])) * dI
        inner = slice(5, n - 5)
        assert np.sign(st[3][inner][np.argmax(np.abs(Vw[inner]))]) == np.sign(Vw[inner][np.argmax(np.abs(Vw[inner]))])
        errs.append(np.max(np.abs(st[3][inner] - Vw[inner])) / np.max(np.abs(Vw[inner])))
    # relative error grows like B^2 (ratio 4 per doubling)
    assert errs[0] < 5e-4
    assert 3.0 < errs[1] / errs[0] < 5.0
    assert 3.0 < errs[2] / errs[1] < 5.0


def test_polarisation_degree_bounded():
    lines = _lines("slit", 64)
    p = _params(300, seed=17)
    st = oracle.me_synth(p, lines)
    pol = np.sqrt(st[:, 1] ** 2 + st[:, 2] ** 2 + st[:, 3] ** 2)
    assert np.all(pol <= st[:, 0] * (1 + 1e-12))
    # the line-only part too: |x_pol| <= x_0 for K^-1 e
    assert np.all(pol <= (st[:, 0] - p[:, 7][:, None]) * (1 + 1e-12))


def test_azimuth_rotation():
    lines = _lines("slit", 48)
    p = _params(12, seed=21)
    dchi = 33.0
    p2 = p.copy()
    p2[:, 2] += dchi
    a, b = oracle.me_synth(p, lines), oracle.me_synth(p2, lines)
    lin_a = (a[:, 1] + 1j * a[:, 2]) * np.exp(2j * math.radians(dchi))
    lin_b = b[:, 1] + 1j * b[:, 2]
    assert np.max(np.abs(lin_a - lin_b)) < 1e-14
    assert np.max(np.abs(a[:, [0, 3]] - b[:, [0, 3]])) < 1e-14


def test_reflection_symmetries():
    lines = _lines("slit", 65)
    p = _params(10, seed=23)
    p[:, 3] = 0.0
    st = oracle.me_synth(p, lines)
    off = 0
    for ln in lines:
        sl = st[:, :, off:off + ln.nlam]
        rev = sl[:, :, ::-1]
        # the absolute wavelengths start + j step are symmetric about lambda0
        # only to ~1e-12 A, which moves the profiles by ~1e-11 at most
        assert np.max(np.abs(sl[:, :3] - rev[:, :3])) < 2e-10      # I, Q, U symmetric
        assert np.max(np.abs(sl[:, 3] + rev[:, 3])) < 2e-10        # V antisymmetric
        off += ln.nlam
    # (gamma, chi) -> (180 - gamma, -chi): I, Q unchanged, U and V flip sign
    q = _params(10, seed=29)
    q2 = q.copy()
    q2[:, 1] = 180.0 - q[:, 1]
    q2[:, 2] = -q[:, 2]
    a, b = oracle.me_synth(q, lines), oracle.me_synth(q2, lines)
    assert np.max(np.abs(a[:, :2] - b[:, :2])) < 1e-13
    assert np.max(np.abs(a[:, 2:] + b[:, 2:])) < 1e-13
    # gamma = 0: Q = U = 0 ; gamma = 90: V = 0
    q3 = q.copy()
    q3[:, 1] = 0.0
    assert np.max(np.abs(oracle.me_synth(q3, lines)[:, 1:3])) < 1e-15
    q3[:, 1] = 90.0
    assert np.max(np.abs(oracle.me_synth(q3, lines)[:, 3])) < 1e-15


def test_mu_scaling():
    lines = _lines("tiny")
    p = _params(5, seed=31)
    mu = np.array([1.0, 0.5, 0.3, 0.9, 0.1])
    st = oracle.me_synth(p, lines, mu)
    s1 = oracle.me_synth(p, lines)
    # I - S0 and Q, U, V scale linearly with mu
    assert np.allclose(st[:, 0] - p[:, 7:8], mu[:, None] * (s1[:, 0] - p[:, 7:8]), atol=1e-15)
    assert np.allclose(st[:, 1:], mu[:, None, None] * s1[:, 1:], atol=1e-15)


def test_chi2_definition():
    lines = _lines("tiny")
    p = _params(3, seed=37)
    st = oracle.me_synth(p, lines)
    L = st.shape[-1]
    sig = si.sigma_for(p)
    obs = st + 1e-3 * si.std_normal(st.shape, 1)
    par = p[:, None, :]
    c = oracle.chi2(par, obs, sig, lines)
    # truth model: chi2 = sum(noise^2 / sigma^2) / (4L - 9)
    ref = np.sum(((obs - st) / sig[:, :, None]) ** 2, axis=(1, 2)) / (4 * L - 9)
    assert np.allclose(c[:, 0], ref, rtol=1e-13)
    assert np.all(oracle.chi2(par, st, sig, lines) < 1e-25)


# --------------------------------------------------------------------------- #
# Decode and the random stream (Sec. 3, Sec. 4.2)

def test_decode_endpoints():
    lo, hi = si.PRIOR_LO, si.PRIOR_HI
    assert np.array_equal(oracle.decode(np.zeros(9, np.uint16), lo, hi), lo)
    assert np.array_equal(oracle.decode(np.full(9, 65535, np.uint16), lo, hi), hi)
    mid = oracle.decode(np.full(9, 32768, np.uint16), lo, hi)
    assert np.allclose(mid, lo + (hi - lo) * 32768 / 65535, rtol=1e-15)


def test_philox_known_answers(golden_dir):
    for row in read_table(os.path.join(golden_dir, "philox4x32_10_kat.txt")):
        vals = [int(x, 16) for x in row]
        out = oracle.philox4x32_10(vals[0:4], vals[4:6])
        assert list(out) == vals[6:10]


def test_rng_word_layout():
    # word n of stream (seed, pixel, gen, indiv, purpose) = Philox(ctr, key)[n % 4]
    seed = (7 << 32) | 12345
    for n in (0, 1, 2, 3, 4, 9, 71):
        ctr = [3, 5, 11, (3 << 24) | (n // 4)]
        assert oracle.rng_word(seed, 3, 5, 11, 3, n) == oracle.philox4x32_10(ctr, [12345, 7])[n % 4]
