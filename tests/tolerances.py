"""Parity bounds shared by the GPU tests (derivations in their docstrings)."""
import numpy as np

# forward model: FP32 within 1e-5 Ic at every sample, FP64 within 1e-10 Ic
FWD_TOL_F32 = 1e-5
FWD_TOL_F64 = 1e-10


def ic_of(p, mu=None):
    """Continuum intensity S0 + mu S1 of parameter rows [..., 9]."""
    m = 1.0 if mu is None else mu
    return p[..., 7] + m * p[..., 8]


def chi2_tol(obs, ref_model, sig, ic, nu, delta_rel):
    """|chi2_gpu - chi2_ref| bound from a forward-model error delta = delta_rel Ic
    at every sample: (1/nu) sum w^2 (2 |r| delta + delta^2) over [npix, pop]."""
    r = np.abs(obs[:, None] - ref_model)
    w2 = 1.0 / sig[:, None, :, None] ** 2
    d = delta_rel * ic[:, None, None, None]
    return (w2 * (2 * r * d + d * d)).sum(axis=(2, 3)) / nu


def recover_genes(params, lo, hi):
    """The 16-bit codes whose decoding (Sec. 3) rounded to float32 gives the
    float32 parameters [n, 9]: p = lo + (hi - lo) g / 65535 is inverted and
    rounded; exact while |p| / (hi - lo) < 127, which holds for every box here."""
    p = np.asarray(params, np.float64)
    g = np.rint((p - lo) / (hi - lo) * 65535.0)
    return np.clip(g, 0, 65535).astype(np.uint16)
