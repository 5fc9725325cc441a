"""FP64 oracle of the heuristic first guesses (Sec. 5.5 seeds the initial
population with field estimates from the weak-field approximation, the
centre-of-gravity method and the observed profile's shape; the formulas below
are this package's readings, written from those approximations).

TEST INFRASTRUCTURE ONLY, like the rest of this package: plain numpy in
float64, one pixel at a time.

Per line, with x_j the sample offsets from the rest wavelength lambda0,
I_c the largest I sample of the pixel (all lines), d_j = I_c - I_j,
d+-_j = I_c - (I_j +- V_j), I' and I'' central differences (one-sided first
differences and I'' = 0 at the window ends), C = 4.6686e-13 lambda0^2 and
gbar the first moment of the line's red sigma group:
  centre of gravity  x_cog = sum x d / sum d  ->  v_los = c x_cog / lambda0;
  longitudinal field (centre of gravity of I + V and I - V)
                     B_par = (x_cog(d+) - x_cog(d-)) / (2 C gbar);
  transverse field (weak-field second-order Q, U = -(1/4) C^2 gbar^2 B_perp^2
                     (cos 2chi, sin 2chi) I'', least squares over the samples)
                     q = -4 sum Q I'' / (C^2 gbar^2 sum I''^2), u likewise;
  half-depth width   hw = step #{j : d_j >= max d / 2} / 2 (half the width
                     of the samples at or above half depth);
  core depth         D = 1 - min I / I_c.
Lines are combined with their equivalent widths W = step sum d as weights
(times gbar for B_par, gbar^2 for q and u).  Then B_perp = sqrt(hypot(q, u)),
azimuth = atan2(u, q)/2, B = hypot(B_par, B_perp), inclination =
atan2(B_perp, B_par); with the source function split S1 mu = 3/4 I_c,
S0 = I_c / 4, eta0 = D'/(1 - D') for D' = min(D / 0.75, 0.97); the Doppler
width from the W-weighted half-depth width: for S0 = 0 the depth 1 - 1/(1 +
eta0 H) falls to half its centre value where H = 1/(eta0 + 2), at
x = dlambda_D sqrt(ln(eta0 + 2)) for a Gaussian core, so dlambda_D =
hw / sqrt(ln(eta0 + 2)); damping the middle of its range; a non-finite
estimate becomes the middle of its range; every value clamped into the
search box (the azimuth wrapped into [0, 180)).
"""
from __future__ import annotations

import numpy as np

C_KMS = 299792.458
ZEEMAN = 4.6686e-13


def gbar_of(line):
    """First moment of the red sigma group of a line's Zeeman pattern."""
    q = np.asarray(line.q[:line.ncomp])
    s = np.asarray(line.shift[:line.ncomp])
    w = np.asarray(line.strength[:line.ncomp])
    r = q == 1
    return float((w[r] * s[r]).sum())


def _derivs(I, step):
    n = len(I)
    d1 = np.empty(n)
    d1[1:-1] = (I[2:] - I[:-2]) / (2 * step)
    d1[0] = (I[1] - I[0]) / step
    d1[-1] = (I[-1] - I[-2]) / step
    d2 = np.zeros(n)
    d2[1:-1] = (I[2:] - 2 * I[1:-1] + I[:-2]) / step ** 2
    return d1, d2


def first_guess(obs, lines, lo, hi, mu=None):
    """obs [npix, 4, L] (the lines' samples concatenated), oracle lines (with
    their grids) -> first guesses [npix, 9]."""
    obs = np.asarray(obs, np.float64)
    npix = obs.shape[0]
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    mus = np.ones(npix) if mu is None else np.broadcast_to(np.asarray(mu, np.float64), (npix,))
    out = np.empty((npix, 9))
    for p in range(npix):
        I_all = obs[p, 0]
        Ic = I_all.max()
        off = 0
        acc = dict(W=0.0, Wv=0.0, Wg=0.0, WgB=0.0, Wg2=0.0, Wq=0.0, Wu=0.0, Wdop=0.0)
        depth = 0.0
        for ln in lines:
            n = ln.nlam
            I, Q, U, V = (obs[p, s, off:off + n] for s in range(4))
            off += n
            x = (ln.start - ln.lambda0) + ln.step * np.arange(n)
            d = Ic - I
            dp = Ic - (I + V)
            dm = Ic - (I - V)
            d1, d2 = _derivs(I, ln.step)
            C = ZEEMAN * ln.lambda0 ** 2
            g = gbar_of(ln)
            s0 = d.sum()
            xc = (x * d).sum() / s0
            v = C_KMS * xc / ln.lambda0
            bpar = ((x * dp).sum() / dp.sum() - (x * dm).sum() / dm.sum()) / (2 * C * g)
            s2 = (d2 * d2).sum()
            q = -4 * (Q * d2).sum() / (C * C * g * g * s2)
            u = -4 * (U * d2).sum() / (C * C * g * g * s2)
            hw = 0.5 * ln.step * np.count_nonzero(d >= 0.5 * d.max())
            W = ln.step * s0
            acc["W"] += W
            acc["Wv"] += W * v
            acc["Wg"] += W * g
            acc["WgB"] += W * g * bpar
            acc["Wg2"] += W * g * g
            acc["Wq"] += W * g * g * q
            acc["Wu"] += W * g * g * u
            acc["Wdop"] += W * hw
            depth = max(depth, 1.0 - I.min() / Ic)
        vlos = acc["Wv"] / acc["W"]
        bpar = acc["WgB"] / acc["Wg"]
        q = acc["Wq"] / acc["Wg2"]
        u = acc["Wu"] / acc["Wg2"]
        bperp = np.sqrt(np.hypot(q, u))
        azim = np.degrees(0.5 * np.arctan2(u, q)) % 180.0
        B = np.hypot(bpar, bperp)
        incl = np.degrees(np.arctan2(bperp, bpar))
        Dp = min(depth / 0.75, 0.97)
        eta0 = Dp / (1.0 - Dp)
        dop = acc["Wdop"] / acc["W"] / np.sqrt(np.log(eta0 + 2.0))
        S1 = 0.75 * Ic / mus[p]
        S0 = 0.25 * Ic
        damp = 0.5 * (lo[5] + hi[5])
        g9 = np.array([B, incl, azim, vlos, dop, damp, eta0, S0, S1])
        g9 = np.where(np.isfinite(g9), g9, 0.5 * (lo + hi))
        g9 = np.minimum(np.maximum(g9, lo), hi)
        out[p] = g9
    return out


# --------------------------------------------------------------------------- #
# The separate seeds of Sec. 5.5

SEED_NAMES = ("weak_field", "integral", "centre_of_gravity", "non_magnetic")


def _thermo(obs_p, lines, lo, hi, mu):
    """v_los, Doppler width, damping, eta0, S0, S1 of first_guess (the
    centre of gravity, half-depth width and core depth estimates)."""
    return first_guess(obs_p[None], lines, lo, hi, mu=np.array([mu]))[0][3:]


def seeds(obs, lines, lo, hi, mu=None, box=None):
    """The four first guesses of Sec. 5.5 per pixel: [npix, 4, 9] in the
    order of SEED_NAMES; a NaN entry is a parameter the seed leaves random.
    Shared by all four: the thermodynamic estimates of first_guess.  Per
    line (x, I_c, I', I'', C, gbar as in first_guess; a = C^2 gbar^2):
      weak field (Auer et al.): the least squares of the weak-field relations
        V = -C gbar B_par I' and (Q, U) = -(1/4) a B_perp^2 (cos 2chi,
        sin 2chi) I'' over the samples of every line:
        B_par = -sum V I' C gbar / sum (C gbar I')^2,
        q = -4 sum a Q I'' / sum (a I'')^2 (u likewise), B_perp =
        sqrt(hypot(q, u)), chi = atan2(u, q) / 2;
      integral relations (Ronan et al.): the same relations integrated over
        the profiles, |B_par| = sum |V| / sum C gbar |I'|, with the sign of
        -sum V I' (the order of the V lobes), B_perp^2 = 4 sum sqrt(Q^2 +
        U^2) / sum a |I''|; the azimuth from the integrated second moments of
        the linear polarisation, whose principal axis is chi0 = atan2(2 sum
        Q U, sum (Q^2 - U^2)) / 4 (Q, U ~ cos 2chi, sin 2chi at every sample
        when magneto-optical mixing is small), chi0 or chi0 + 90 deg: the one
        whose projection Q cos 2chi + U sin 2chi summed over the three samples
        around each line's minimum of I is not positive (at the line centre
        the pi component gives Q ~ -cos 2chi);
      centre of gravity (Rees and Semel): B = |B_par| of first_guess's
        centre-of-gravity estimate, inclination 0 for B_par >= 0 and 180
        otherwise, azimuth unseeded;
      non-magnetic: B = 0, both angles unseeded.
    For the first three, B = hypot(B_par, B_perp) and inclination =
    atan2(B_perp, B_par).  Every seed is then made consistent with the
    pixel's box (box [npix, 2, 9], e.g. the polarity restriction): an
    inclination outside the box's range becomes 180 - inclination; then
    every seeded value is clamped into the box (the azimuth wrapped into
    [0, 180) first); a non-finite estimate is replaced by the middle of the
    box."""
    obs = np.asarray(obs, np.float64)
    npix = obs.shape[0]
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    mus = np.ones(npix) if mu is None else np.broadcast_to(np.asarray(mu, np.float64), (npix,))
    comb = first_guess(obs, lines, lo, hi, mu=mus)
    out = np.full((npix, 4, 9), np.nan)
    for p in range(npix):
        blo = lo if box is None else np.asarray(box[p, 0], np.float64)
        bhi = hi if box is None else np.asarray(box[p, 1], np.float64)
        Ic = obs[p, 0].max()
        off = 0
        s = dict(vI=0.0, I2=0.0, aQ=0.0, aU=0.0, a2=0.0, absV=0.0, absI1=0.0, L=0.0, absI2=0.0,
                 QU=0.0, QQUU=0.0, cQ=0.0, cU=0.0)
        for ln in lines:
            n = ln.nlam
            I, Q, U, V = (obs[p, k, off:off + n] for k in range(4))
            off += n
            d1, d2 = _derivs(I, ln.step)
            C = ZEEMAN * ln.lambda0 ** 2
            g = gbar_of(ln)
            cg = C * g
            a = cg * cg
            s["vI"] += (V * d1).sum() * cg
            s["I2"] += ((cg * d1) ** 2).sum()
            s["aQ"] += a * (Q * d2).sum()
            s["aU"] += a * (U * d2).sum()
            s["a2"] += ((a * d2) ** 2).sum()
            s["absV"] += np.abs(V).sum()
            s["absI1"] += cg * np.abs(d1).sum()
            s["L"] += np.sqrt(Q * Q + U * U).sum()
            s["absI2"] += a * np.abs(d2).sum()
            s["QU"] += (Q * U).sum()
            s["QQUU"] += (Q * Q - U * U).sum()
            c = int(np.argmin(I))
            s["cQ"] += Q[max(c - 1, 0):c + 2].sum()
            s["cU"] += U[max(c - 1, 0):c + 2].sum()
        th = comb[p, 3:]
        cb = _cog_bpar(obs[p], lines)
        # weak field
        bpar = -s["vI"] / s["I2"]
        q = -4.0 * s["aQ"] / s["a2"]
        u = -4.0 * s["aU"] / s["a2"]
        bperp = np.sqrt(np.hypot(q, u))
        wf = [np.hypot(bpar, bperp), np.degrees(np.arctan2(bperp, bpar)),
              np.degrees(0.5 * np.arctan2(u, q))]
        # integral relations
        ipar = np.abs(s["absV"] / s["absI1"]) * (1.0 if -s["vI"] >= 0 else -1.0)
        iperp = np.sqrt(4.0 * s["L"] / s["absI2"])
        chi0 = 0.25 * np.arctan2(2.0 * s["QU"], s["QQUU"])
        if s["cQ"] * np.cos(2 * chi0) + s["cU"] * np.sin(2 * chi0) > 0:
            chi0 += 0.5 * np.pi
        ir = [np.hypot(ipar, iperp), np.degrees(np.arctan2(iperp, ipar)), np.degrees(chi0)]
        # centre of gravity: the longitudinal estimate of first_guess
        cog = [abs(cb), 0.0 if cb >= 0 else 180.0, np.nan]
        for k, mag in enumerate((wf, ir, cog, [0.0, np.nan, np.nan])):
            v = np.concatenate([np.asarray(mag, np.float64), th])
            out[p, k] = _consistent(v, blo, bhi)
    return out


def _cog_bpar(obs_p, lines):
    """first_guess's centre-of-gravity longitudinal field of one pixel: the
    per-line estimates (x_cog(d+) - x_cog(d-)) / (2 C gbar) combined with the
    weights W gbar."""
    Ic = obs_p[0].max()
    off = 0
    Wg = WgB = 0.0
    for ln in lines:
        n = ln.nlam
        I, V = obs_p[0, off:off + n], obs_p[3, off:off + n]
        off += n
        x = (ln.start - ln.lambda0) + ln.step * np.arange(n)
        d = Ic - I
        dp = Ic - (I + V)
        dm = Ic - (I - V)
        C = ZEEMAN * ln.lambda0 ** 2
        g = gbar_of(ln)
        bpar = ((x * dp).sum() / dp.sum() - (x * dm).sum() / dm.sum()) / (2 * C * g)
        W = ln.step * d.sum()
        Wg += W * g
        WgB += W * g * bpar
    return WgB / Wg


def _consistent(v, blo, bhi):
    """Polarity consistency, azimuth wrap, non-finite -> middle, clamp (NaN
    angles stay unseeded)."""
    v = v.copy()
    seeded = ~np.isnan(v)
    seeded[0] = True
    v[0] = v[0] if np.isfinite(v[0]) else 0.5 * (blo[0] + bhi[0])
    for j in (1, 2):
        if seeded[j] and not np.isfinite(v[j]):
            v[j] = 0.5 * (blo[j] + bhi[j])
    if seeded[2]:
        v[2] = v[2] % 180.0
    if seeded[1] and not (blo[1] <= v[1] <= bhi[1]):
        v[1] = 180.0 - v[1]
    for j in range(3, 9):
        if not np.isfinite(v[j]):
            v[j] = 0.5 * (blo[j] + bhi[j])
    return np.where(seeded, np.minimum(np.maximum(v, blo), bhi), np.nan)
