"""Inverse-max weighting of the merit function (Sec. 5.4), FP64.

TEST INFRASTRUCTURE ONLY: the plain definition the HIP path is checked against.

Sec. 5.4 weights each Stokes parameter of a pixel by the inverse of its
largest observed signal, so that I, Q, U and V count about equally in the
chi-square of Sec. 5 (whose weights are constant over the line):
w_I = 1 / (I_c - I_0) with I_c the continuum and I_0 the line-core intensity,
w_Q = 1 / max |Q|, w_U = 1 / max |U|, w_V = 1 / max |V|.  The chi-square
takes sigma = 1 / w.  Readings where the section is silent: I_c is the
largest and I_0 the smallest observed I over every sample of the pixel (all
lines together), and each sigma is at least `floor` (a Stokes parameter with
no signal, Q = U = V = 0 at zero field, would otherwise get an infinite
weight).  A non-finite sample makes the pixel's four sigmas NaN.
"""
from __future__ import annotations

import numpy as np


def invmax_sigma(obs, floor):
    """sigma [npix, 4] = 1 / w of Sec. 5.4 for observations [npix, 4, L]."""
    obs = np.asarray(obs, dtype=np.float64)
    npix = obs.shape[0]
    out = np.empty((npix, 4))
    for p in range(npix):
        I, Q, U, V = obs[p]
        if not np.all(np.isfinite(obs[p])):
            out[p] = np.nan
            continue
        amp = [max(I) - min(I), max(abs(Q)), max(abs(U)), max(abs(V))]
        out[p] = [max(a, floor) for a in amp]
    return out
