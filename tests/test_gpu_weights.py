"""Inverse-max weights of Sec. 5.4 on the GPU (me_invmax_sigma, FP32 and
FP64) against the oracle's definition: bit-exact (max, min and |.| are exact;
the one subtraction of two samples of the same precision is done exactly in
FP64 by the oracle and correctly rounded on both sides), over several tiles of
pixels with ragged sample counts, zero polarisation, a non-finite sample and
the empty input; and a GA inversion under these weights whose best chi-square
is the oracle's chi-square of the returned parameters with the same weights."""
import numpy as np
import pytest
import torch

import oracle
from oracle import weights as ow
import synth_inputs as si
from conftest import gpu_available
from tolerances import FWD_TOL_F32, chi2_tol, ic_of

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"
LO, HI = si.PRIOR_LO, si.PRIOR_HI


def _setup(kind):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set(kind):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    return lines, grids, olines


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["slit", "tiny"])
def test_invmax_sigma_bit_exact(kind, dtype):
    lines, grids, olines = _setup(kind)
    n = 517
    truth = si.draw_truth(n, 41)
    truth[:7, 0] = 0.0                       # no polarisation: the floor
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 41)
    obs[:3, 1:] = 0.0
    obs[9, 2, 5] = np.nan
    obs[10, 0, 0] = np.inf
    npd = np.float32 if dtype == torch.float32 else np.float64
    o = obs.astype(npd)
    floor = 3e-4
    got = g.me_invmax_sigma(torch.tensor(o, device=DEV), grids, floor).cpu().numpy()
    ref = ow.invmax_sigma(o.astype(np.float64), float(npd(floor))).astype(npd)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    assert np.all(np.isnan(got[9])) and np.all(np.isnan(got[10]))
    assert np.all(got[:3, 1:] == npd(floor))
    e = g.me_invmax_sigma(torch.zeros((0, 4, o.shape[2]), dtype=dtype, device=DEV), grids)
    assert e.shape == (0, 4)
    with pytest.raises(g.GenesisError):
        g.me_invmax_sigma(torch.tensor(o, device=DEV), grids, -1.0)


def test_inversion_under_invmax_weights():
    lines, grids, olines = _setup("slit")
    n = 96
    truth = si.draw_truth(n, 42)
    obs = oracle.me_synth(truth, olines)
    o32 = torch.tensor(obs, dtype=torch.float32, device=DEV)
    s32 = g.me_invmax_sigma(o32, grids, 1e-4)
    res = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI),
                      g.GAConfig(pop=64, generations=40, seed=5))
    bp = res["params"].double().cpu().numpy()
    s64 = s32.double().cpu().numpy()
    o64 = o32.double().cpu().numpy()
    c_or = oracle.chi2(bp[:, None, :], o64, s64, olines)[:, 0]
    c_gpu = res["chi2"].double().cpu().numpy()
    assert np.all(res["status"].cpu().numpy() == 0)
    # the FP32 forward model is within 1e-5 Ic of the oracle's at every
    # sample; the bound that puts on the chi-square, plus FP32 accumulation
    models = oracle.me_synth(bp, olines)[:, None]
    tol = chi2_tol(o64, models, s64, ic_of(bp), 4 * obs.shape[2] - 9, FWD_TOL_F32)[:, 0]
    assert np.all(np.abs(c_gpu - c_or) <= tol + 8e-5 * c_or)
