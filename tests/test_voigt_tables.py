"""The generated rational approximations of the Faddeeva function that the HIP
kernels compile in (voigt_rational.h for FP32, voigt_rational_h.h for the
packed-FP16 synthesis), checked on the CPU against scipy.special.wofz.

w(z) = exp(-z^2) erfc(-iz) at z = v + i a is approximated by P(Z)/Q(Z) with
Z = a - i v.  The stated maximum error holds on a = 0; the denominator's
zeros lie in Re Z < 0, so P/Q - w is analytic in a >= 0 and the bound holds
for every damping (maximum modulus).  For the FP16 path the per-individual
polynomials in the compact variable t = 1/(1 + v^2/2), scaled by
1/sqrt(D~(0) D~(1)), must keep every coefficient small for damping in [0, 1]
(at most 4.3 in magnitude, so FP16 rounds each one by at most 2e-3), and
still reproduce w."""
import os
import re
from math import comb

import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

wofz = pytest.importorskip("scipy.special").wofz

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1208_0302_amd", "csrc")


def _table(name, pre):
    text = open(os.path.join(CSRC, name)).read()

    def block(tag, nxt):
        a = text.index("#define %s_%s" % (pre, tag))
        b = text.index(nxt, a + 1) if nxt else len(text)
        return [float(x) for x in re.findall(r"[-+]?\d\.\d+e[-+]\d+", text[a:b])]

    p = np.array(block("P_INIT", "#define %s_Q_INIT" % pre))
    q = np.array(block("Q_INIT", None))
    np_ = int(re.search(r"#define %s_NP (\d+)" % pre, text).group(1))
    nq = int(re.search(r"#define %s_NQ (\d+)" % pre, text).group(1))
    maxerr = float(re.search(r"#define %s_MAXERR (\S+)" % pre, text).group(1))
    assert len(p) == np_ and len(q) == nq
    return p, q, maxerr


TABLES = [("voigt_rational.h", "GENESIS_VR", 2e-7), ("voigt_rational_h.h", "GENESIS_VRH", 2e-4)]


@pytest.mark.parametrize("name,pre,bound", TABLES)
def test_rational_error_bound(name, pre, bound):
    p, q, maxerr = _table(name, pre)
    assert maxerr <= bound
    v = np.concatenate([np.linspace(-60, 60, 48001), np.geomspace(60, 1e4, 400),
                        -np.geomspace(60, 1e4, 400)])
    worst = 0.0
    for a in (0.0, 1e-3, 0.01, 0.05, 0.1, 0.3, 0.5, 1.0, 1.5, 3.0, 10.0):
        Z = a - 1j * v
        r = np.polyval(p[::-1], Z) / np.polyval(q[::-1], Z)
        worst = max(worst, np.abs(r - wofz(v + 1j * a)).max())
    assert worst <= maxerr * 1.001 + 1e-15, (worst, maxerr)
    # the bound is attained on the real axis, not just below it
    assert worst >= 0.5 * maxerr


@pytest.mark.parametrize("name,pre,bound", TABLES)
def test_denominator_is_stable(name, pre, bound):
    p, q, _ = _table(name, pre)
    assert q[0] == 1.0
    assert np.roots(q[::-1]).real.max() < 0.0
    # leading ratio 1/sqrt(pi): w ~ 1/(sqrt(pi) Z) at infinity
    assert p[-1] / q[-1] == pytest.approx(1.0 / np.sqrt(np.pi), rel=1e-12)


def _shift(c, a):
    # coefficients of c(x + a)
    return np.array([sum(comb(m, k) * c[m] * a ** (m - k) for m in range(k, len(c)))
                     for k in range(len(c))])


def _compact(p, q, a, s=2.0):
    pp, qq = _shift(p, a), _shift(q, a)
    sg = lambda m: -1.0 if m & 1 else 1.0
    ep = np.array([sg(m) * pp[2 * m] for m in range((len(pp) + 1) // 2)])
    op = np.array([sg(m) * pp[2 * m + 1] for m in range(len(pp) // 2)])
    eq = np.array([sg(m) * qq[2 * m] for m in range((len(qq) + 1) // 2)])
    oq = np.array([sg(m) * qq[2 * m + 1] for m in range(len(qq) // 2)])
    nh = Pn.polyadd(Pn.polymul(ep, eq), np.concatenate([[0.0], Pn.polymul(op, oq)]))
    nl = Pn.polysub(Pn.polymul(ep, oq), Pn.polymul(op, eq))
    d = Pn.polyadd(Pn.polymul(eq, eq), np.concatenate([[0.0], Pn.polymul(oq, oq)]))
    n = len(q) - 1

    def to_t(c):
        out = np.zeros(n + 1)
        for k, ck in enumerate(c):
            term = ck * s ** k * Pn.polypow([1.0, -1.0], k)
            term = Pn.polymul(term, np.eye(1, n - k + 1, n - k)[0])
            out[:len(term)] += term
        return out

    th, tl, td = to_t(nh), to_t(nl), to_t(d)
    k = 1.0 / np.sqrt(td[0] * td.sum())
    return th * k, tl * k, td * k


def test_fp16_compact_coefficients_are_small():
    p, q, _ = _table("voigt_rational_h.h", "GENESIS_VRH")
    hi = 0.0
    for a in np.linspace(0.0, 1.0, 201):
        th, tl, td = _compact(p, q, a)
        hi = max(hi, np.abs(np.concatenate([th, tl, td])).max())
        # the compact form still gives the Faddeeva function
        v = np.linspace(-40, 40, 2001)
        t = 1.0 / (1.0 + v * v / 2.0)
        H = np.polyval(th[::-1], t) / np.polyval(td[::-1], t)
        L = v * np.polyval(tl[::-1], t) / np.polyval(td[::-1], t)
        w = wofz(v + 1j * a)
        assert np.abs(H - w.real).max() < 2e-4 and np.abs(L - w.imag).max() < 2e-4
    assert hi <= 4.3, hi


@pytest.mark.parametrize("n,name,pre", [(7, "voigt_rational.h", "GENESIS_VR"),
                                        (4, "voigt_rational_h.h", "GENESIS_VRH")])
def test_tables_come_from_the_generator(n, name, pre):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "gen_voigt_rational", os.path.join(CSRC, "gen_voigt_rational.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    m, p, q = gen.fit(n)
    ph, qh, mh = _table(name, pre)
    assert np.allclose(p, ph, rtol=1e-9, atol=0) and np.allclose(q, qh, rtol=1e-9, atol=0)
    assert m == pytest.approx(mh, rel=1e-5)


@pytest.mark.parametrize("n, bound", [(36, 1e-13), (28, 3e-12)])
def test_weideman_table_of_the_fp64_kernels(n, bound):
    # w(z) = r (2 p(Z) r + 1/sqrt(pi)), r = 1/(L - i z), Z = (L + i z) r,
    # p(Z) = sum c_n Z^n (Weideman 1994), as the FP64 kernels evaluate it:
    # N = 36 for the forward model, the search and the refinement, N = 28 for
    # the uncertainty kernel's merit function
    text = open(os.path.join(CSRC, "weideman%d.h" % n)).read()
    WL = float(re.search(r"#define GENESIS_WD%d_L (\S+)" % n, text).group(1))
    c = np.array([float(x) for x in
                  re.findall(r"[-+]?\d\.\d+e[-+]\d+",
                             text[text.index("genesis_wd%d_c" % n):])])
    assert len(c) == n
    worst = 0.0
    v = np.linspace(-60, 60, 24001)
    for a in (0.0, 1e-4, 0.01, 0.1, 0.5, 1.0, 2.0, 5.0):
        z = v + 1j * a
        r = 1.0 / (WL - 1j * z)
        Z = (WL + 1j * z) * r
        p = np.polyval(c[::-1], Z)
        w = r * (2.0 * p * r + 1.0 / np.sqrt(np.pi))
        worst = max(worst, np.abs(w - wofz(z)).max())
    assert worst < bound, worst
