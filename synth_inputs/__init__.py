"""Seeded synthetic inputs shared by the oracle tests, the HIP tests and the
benchmark.

This module holds line data, wavelength grids, parameter priors and random
draws only.  It contains none of the inversion method's arithmetic (no Zeeman
pattern, no profile, no synthesis, no genetic operator): the forward model that
turns truth parameters into observed Stokes profiles lives on each side of the
comparison separately.

Line data are Fe I multiplet 816 of Table 1 (Sec. 2).  Lande factors are the
LS-coupling values of the listed terms: 5P2 = 11/6, 5D2 = 3/2, 5P1 = 5/2,
5D0 has J = 0.  The lower level is the 5P term.

Priors follow the synthetic workloads used throughout the tests and the
benchmark: B U(0, 3000) G, inclination U(0, 180) deg, azimuth U(0, 180) deg,
v_los N(0, 1.5) km/s clipped to +-7.5, Doppler width U(20, 50) mA, damping
U(0, 0.5), eta0 U(1, 30), S0 U(0, 0.5), S1 U(0.5, 1); noise sigma = 1e-3 Ic
with Ic = S0 + mu S1.
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("B", "incl", "azim", "vlos", "dopp", "damp", "eta0", "S0", "S1")
NPAR = 9

# GA search box = prior box (v_los box at +-5 sigma of its normal prior)
PRIOR_LO = np.array([0.0, 0.0, 0.0, -7.5, 0.020, 0.0, 1.0, 0.0, 0.5])
PRIOR_HI = np.array([3000.0, 180.0, 180.0, 7.5, 0.050, 0.5, 30.0, 0.5, 1.0])

# Table 1 lines: rest wavelength [A] and (J, g) of lower and upper level
FE6301 = dict(name="FeI6301.5", lambda0=6301.5091, Jl=2.0, gl=11.0 / 6.0, Ju=2.0, gu=1.5,
              terms=((2, 1, 2), (2, 2, 2)))   # (S, L, J) of lower, upper
FE6302 = dict(name="FeI6302.5", lambda0=6302.5017, Jl=1.0, gl=2.5, Ju=0.0, gu=0.0,
              terms=((2, 1, 1), (2, 2, 0)))
TABLE1_GEFF = {"FeI6301.5": 1.667, "FeI6302.5": 2.500}


def grid(line: dict, nlam: int, half_width: float = 0.4):
    """Wavelength grid of one line: nlam samples over lambda0 +- half_width,
    end points included.  Returns (start, step) in Angstrom."""
    start = line["lambda0"] - half_width
    step = 2.0 * half_width / (nlam - 1)
    return start, step


def line_set(name: str):
    """Named line/grid sets of the synthetic workloads:
    'tiny'  -- one line (6302.5) x 100 samples;
    'slit'  -- both lines x 128 samples."""
    if name == "tiny":
        return [(FE6302, 100)]
    if name == "slit":
        return [(FE6301, 128), (FE6302, 128)]
    if name == "slit1":
        return [(FE6302, 128)]
    raise KeyError(name)


# Stand-in for the centre-to-limb variation of the field-free (quiet-Sun)
# Stokes I profile that the fill-fraction model mixes in (Sec. 5.2): the paper
# fits its depth, width and damping with cubic polynomials in mu from
# measurements that are not published.  These coefficients (mu^0 .. mu^3) are
# invented: at disc centre a depth of 0.67 (6301.5) and 0.60 (6302.5) of the
# continuum, Doppler width 0.030 A, damping 0.22, weakening, widening and
# more damped towards the limb.
FILL_CLV = {
    "depth": {"6301": (0.50, 0.25, -0.10, 0.02), "6302": (0.45, 0.22, -0.08, 0.01)},
    "width": {"6301": (0.036, -0.008, 0.002, 0.0), "6302": (0.036, -0.008, 0.002, 0.0)},
    "damp": {"6301": (0.30, -0.10, 0.02, 0.0), "6302": (0.30, -0.10, 0.02, 0.0)},
}


def fill_coefficients(name: str):
    """(depth, width, damp) [nlines, 4] of the stand-in profile for a line set."""
    keys = ["6301" if abs(ln["lambda0"] - FE6301["lambda0"]) < 0.5 else "6302"
            for ln, _ in line_set(name)]
    return tuple(np.array([FILL_CLV[q][k] for k in keys]) for q in ("depth", "width", "damp"))


def draw_alpha(npix: int, seed: int, lo: float = 0.25, hi: float = 1.0) -> np.ndarray:
    """Fill fractions uniform in [lo, hi] (Table 4 bounds alpha below by 0.25
    in umbrae and penumbrae)."""
    return np.random.default_rng(seed + 7777).uniform(lo, hi, npix)


def draw_truth(npix: int, seed: int) -> np.ndarray:
    """Truth parameters [npix, 9] drawn iid from the priors (float64)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    p = np.empty((npix, NPAR))
    p[:, 0] = rng.uniform(0.0, 3000.0, npix)
    p[:, 1] = rng.uniform(0.0, 180.0, npix)
    p[:, 2] = rng.uniform(0.0, 180.0, npix)
    p[:, 3] = np.clip(rng.normal(0.0, 1.5, npix), -7.5, 7.5)
    p[:, 4] = rng.uniform(0.020, 0.050, npix)
    p[:, 5] = rng.uniform(0.0, 0.5, npix)
    p[:, 6] = rng.uniform(1.0, 30.0, npix)
    p[:, 7] = rng.uniform(0.0, 0.5, npix)
    p[:, 8] = rng.uniform(0.5, 1.0, npix)
    return p


def draw_uniform_box(n: int, seed: int, lo=PRIOR_LO, hi=PRIOR_HI) -> np.ndarray:
    """Parameters [n, 9] uniform in a box (used for parity sweeps)."""
    rng = np.random.Generator(np.random.Philox(key=seed + 7919))
    u = rng.uniform(size=(n, NPAR))
    return np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * u


def sigma_for(truth: np.ndarray, mu=None, rel: float = 1e-3) -> np.ndarray:
    """Per-pixel, per-Stokes noise sigma [npix, 4] = rel * (S0 + mu S1)."""
    m = 1.0 if mu is None else np.asarray(mu, np.float64)
    ic = truth[:, 7] + m * truth[:, 8]
    return np.repeat((rel * ic)[:, None], 4, axis=1)


def std_normal(shape, seed: int) -> np.ndarray:
    """Standard-normal draws for additive observation noise."""
    rng = np.random.Generator(np.random.Philox(key=seed + 104729))
    return rng.standard_normal(shape)


def random_genes(npix: int, pop: int, seed: int) -> np.ndarray:
    """Arbitrary 16-bit genotypes [npix, pop, 9] (inputs of operator tests)."""
    rng = np.random.Generator(np.random.Philox(key=seed + 31337))
    return rng.integers(0, 65536, size=(npix, pop, NPAR), dtype=np.uint16)


def random_fitness(npix: int, pop: int, seed: int, ties: bool = True, nans: bool = False):
    """Fitness values [npix, pop] as float32-representable numbers, with
    deliberate ties (and optionally NaNs) so that tie-breaking is exercised."""
    rng = np.random.Generator(np.random.Philox(key=seed + 2718))
    f = rng.gamma(2.0, 1.0, size=(npix, pop)).astype(np.float32)
    if ties:
        idx = rng.integers(0, pop, size=(npix, pop // 4))
        src = rng.integers(0, pop, size=(npix, pop // 4))
        for p in range(npix):
            f[p, idx[p]] = f[p, src[p]]
    if nans:
        idx = rng.integers(0, pop, size=(npix, max(1, pop // 16)))
        for p in range(npix):
            f[p, idx[p]] = np.nan
    return f.astype(np.float64)


def disc_mask(n: int = 2048, radius: float = 1024.0) -> np.ndarray:
    """Boolean on-disc mask of an n x n grid, centre ((n-1)/2, (n-1)/2)."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n]
    return (x - c) ** 2 + (y - c) ** 2 <= radius ** 2


def serving_schedule(rate_per_s: float, window_s: float, seed: int, median_px: float = 4096.0,
                     min_px: int = 256, max_px: int = 65536):
    """Poisson arrivals at `rate_per_s` over `window_s` seconds.  Each request:
    tile pixels clip(lognormal(ln median_px, 1.2), min_px, max_px) (by default
    the serving configuration's 4096, 256, 65536), one line (6302.5) or both
    lines with probability 1/2 each, generations uniform in 50..300.
    Returns a list of dicts (t, npix, lines, generations, seed)."""
    rng = np.random.Generator(np.random.Philox(key=seed + 424242))
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t > window_s:
            break
        npix = int(np.clip(np.round(rng.lognormal(np.log(median_px), 1.2)), min_px, max_px))
        lines = "slit" if rng.uniform() < 0.5 else "slit1"
        gens = int(rng.integers(50, 301))
        out.append(dict(t=t, npix=npix, lines=lines, generations=gens, seed=seed * 100003 + i))
        i += 1
    return out


def full_disc(n: int = 2048, seed: int = 0, corr_px: float = 20.0, strong_frac: float = 0.01,
              stride: int = 1):
    """Full-disc parameter maps: every parameter is a smooth random field
    (white noise filtered by a Gaussian of `corr_px` pixels, rescaled to unit
    variance, then mapped through the prior: uniform priors by the normal CDF,
    v_los as 1.5 z clipped to +-7.5), plus strong-field patches of B in
    U(1500, 3000) G covering about `strong_frac` of the disc.  Returns
    (params [m, 9], mu [m], (y, x) [m, 2]) for the on-disc pixels of an n x n
    grid (disc radius n/2), keeping every `stride`-th on-disc pixel.
    mu = cos(heliocentric angle) = sqrt(1 - r^2)."""
    from scipy.ndimage import gaussian_filter
    from scipy.special import ndtr
    rng = np.random.Generator(np.random.Philox(key=seed + 8191))
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n]
    r = np.hypot(xx - c, yy - c) / (n / 2.0)
    on = r < 1.0
    fields = np.empty((NPAR, n, n), np.float32)
    for j in range(NPAR):
        z = gaussian_filter(rng.standard_normal((n, n)).astype(np.float32), corr_px,
                            mode="wrap")
        z /= z.std()
        fields[j] = z
    p = np.empty((NPAR, n, n), np.float64)
    for j in range(NPAR):
        if j == 3:
            p[j] = np.clip(1.5 * fields[j], -7.5, 7.5)
        else:
            p[j] = PRIOR_LO[j] + (PRIOR_HI[j] - PRIOR_LO[j]) * ndtr(fields[j])
    # strong-field patches: discs of radius 8..24 px until strong_frac is covered
    strong = np.zeros((n, n), bool)
    target = strong_frac * on.sum()
    while (strong & on).sum() < target:
        cy, cx = rng.uniform(0, n, 2)
        rad = rng.uniform(8, 24)
        m = (yy - cy) ** 2 + (xx - cx) ** 2 <= rad * rad
        p[0][m] = rng.uniform(1500.0, 3000.0)
        strong |= m
    iy, ix = np.nonzero(on)
    iy, ix = iy[::stride], ix[::stride]
    params = p[:, iy, ix].T.copy()
    mu = np.sqrt(np.clip(1.0 - r[iy, ix] ** 2, 0.0, 1.0))
    return params, mu, np.stack([iy, ix], 1)
