"""FP64 oracle of the per-pixel search boxes: the ranges the non-magnetic
pre-fit gives the thermodynamic parameters (Sec. 5.3) and the polarity
restriction of the inclination (Sec. 5.5).  The paper states neither the
ranges nor the test of the lobe order; the rules below are this package's
readings.

TEST INFRASTRUCTURE ONLY, like the rest of this package: plain numpy in
float64, one pixel at a time.

Starting from the common box [lo, hi], per pixel:
  pre-fit values f (when given; a non-finite value, or a non-positive one for
  the multiplicative windows, leaves that range alone), everything clipped
  into [lo, hi]:
    Doppler width  hi = 1.1 f      (a non-magnetic fit absorbs the Zeeman
    damping        hi = 1.5 f + 0.1 (hi - lo)     broadening into these two)
    eta0           [f / 8, 8 f]
    S1 (beta0)     [f / 1.5, 1.5 f]
  polarity (when n_sigma > 0): I_c the largest I of the pixel (all lines);
  per line x_j the sample offsets from lambda0, x_c = sum x (I_c - I) /
  sum (I_c - I); s = sum over lines and samples of (x_j - x_c) V_j and
  q = sum (x_j - x_c)^2.  V's first moment is negative below 90 degrees of
  inclination (Unno-Rachkovsky: V follows -cos(incl) dI/dlambda), so when
  |s| > n_sigma sigma_V sqrt(q) the inclination range is intersected with
  [0, 90] (s < 0) or [90, 180] (s > 0), unless the intersection is empty.
"""
from __future__ import annotations

import numpy as np


def search_box(obs, sigma, lines, lo, hi, prefit=None, n_sigma=3.0):
    """obs [npix, 4, L], sigma [npix, 4], oracle lines (with grids), common box
    lo/hi [9], prefit [npix, 9] or None -> boxes [npix, 2, 9] (lo, hi)."""
    obs = np.asarray(obs, np.float64)
    sigma = np.asarray(sigma, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    npix = obs.shape[0]
    out = np.empty((npix, 2, 9))
    for p in range(npix):
        blo, bhi = lo.copy(), hi.copy()
        if n_sigma > 0:
            I_all, V_all = obs[p, 0], obs[p, 3]
            Ic = I_all.max()
            s = q = 0.0
            off = 0
            for ln in lines:
                n = ln.nlam
                x = (ln.start - ln.lambda0) + ln.step * np.arange(n)
                d = Ic - I_all[off:off + n]
                xc = (x * d).sum() / d.sum()
                s += ((x - xc) * V_all[off:off + n]).sum()
                q += ((x - xc) ** 2).sum()
                off += n
            if abs(s) > n_sigma * sigma[p, 3] * np.sqrt(q):
                if s > 0 and hi[1] >= 90.0:
                    blo[1] = max(lo[1], 90.0)
                elif s < 0 and lo[1] <= 90.0:
                    bhi[1] = min(hi[1], 90.0)
        if prefit is not None:
            f = np.asarray(prefit, np.float64)[p]
            clip = lambda v, j: min(max(v, lo[j]), hi[j])
            if np.isfinite(f[4]):
                bhi[4] = clip(1.1 * f[4], 4)
            if np.isfinite(f[5]):
                bhi[5] = clip(1.5 * f[5] + 0.1 * (hi[5] - lo[5]), 5)
            if np.isfinite(f[6]) and f[6] > 0:
                blo[6], bhi[6] = clip(f[6] / 8.0, 6), clip(f[6] * 8.0, 6)
            if np.isfinite(f[8]) and f[8] > 0:
                blo[8], bhi[8] = clip(f[8] / 1.5, 8), clip(f[8] * 1.5, 8)
        out[p, 0], out[p, 1] = blo, bhi
    return out
