"""Reduced-precision synthesis (packed FP16 profiles, FP32 Unno-Rachkovsky
and chi-square) through the C ABI, against the FP64 oracle.

Tolerance.  The FP16 path evaluates its own degree-4 rational (error 1.5e-4
for every damping); in FP16 the compactified evaluation is good to 4.4e-3 in
H and 2.7e-3 in L (H(0,0) = 1) for damping <= 1, worst case over |v| <= 300
in an FP16-rounding simulation.  Each group profile is a strength-weighted
mean of components (weights summing to 1), so the group profiles carry the
same absolute error; the test prints the deviation it measures in the
Stokes vector.  The per-sample bound used here is 5e-3 Ic,
with an RMS bound of 1e-3 Ic over all samples, and the chi-square against
noisy data must stay within a few per cent of the FP32 path's."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"
TOL_MAX = 5e-3
TOL_RMS = 1e-3


def _setup(kind, nlam=None):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set(kind):
        n = nlam or n
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    return lines, grids, olines


def _params(n, seed):
    p = si.draw_uniform_box(n, seed)
    k = n // 8
    p[:k, 0] = 0.0
    p[k:2 * k, 1] = 0.0
    p[2 * k:3 * k, 1] = 90.0
    p[3 * k:4 * k, 5] = 0.0
    p[4 * k:5 * k, 6] = 30.0
    p[5 * k:6 * k, 0] = 3000.0
    p[5 * k:6 * k, 4] = 0.02
    p[6 * k:7 * k, 5] = 0.5
    return p


@pytest.mark.parametrize("kind,nlam", [("slit", None), ("tiny", None), ("tiny", 101)])
def test_fp16_synthesis_matches_oracle(kind, nlam):
    lines, grids, olines = _setup(kind, nlam)
    p = _params(400, 3)
    mu = np.linspace(0.2, 1.0, 400)
    got = g.me_synth(torch.tensor(p, dtype=torch.float32, device=DEV), lines, grids,
                     mu=torch.tensor(mu, dtype=torch.float32, device=DEV), fp16=True)
    ref = oracle.me_synth(p.astype(np.float32).astype(np.float64), olines, mu=mu)
    ic = (p[:, 7] + mu * p[:, 8])[:, None, None]
    err = np.abs(got.cpu().numpy() - ref) / ic
    assert np.isfinite(err).all()
    print("%s/%s: max %.2e Ic, rms %.2e Ic" % (kind, nlam, err.max(), np.sqrt((err ** 2).mean())))
    assert err.max() <= TOL_MAX, err.max()
    assert np.sqrt((err ** 2).mean()) <= TOL_RMS
    # odd sample counts: the last wavelength is synthesised alone
    assert got.shape[-1] == sum(gr.n for gr in grids)


def test_fp16_damping_edges():
    # damping 0 (pure Doppler core) and 1 (the largest allowed)
    lines, grids, olines = _setup("slit")
    p = _params(64, 9)
    p[:32, 5] = 0.0
    p[32:, 5] = 1.0
    got = g.me_synth(torch.tensor(p, dtype=torch.float32, device=DEV), lines, grids, fp16=True)
    ref = oracle.me_synth(p.astype(np.float32).astype(np.float64), olines)
    ic = (p[:, 7] + p[:, 8])[:, None, None]
    assert (np.abs(got.cpu().numpy() - ref) / ic).max() <= TOL_MAX


def _problem(npix, seed):
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(npix, seed)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return (lines, grids, olines, truth, torch.tensor(obs.astype(np.float32), device=DEV),
            torch.tensor(sig.astype(np.float32), device=DEV))


def test_fp16_loop_fitness_is_its_synthesis():
    # every final fitness of the FP16 loop is the chi-square of me_synth_f16's
    # Stokes vector of the decoded genes (same device synthesis), and within
    # the synthesis tolerance of the FP64 oracle's chi-square
    lines, grids, olines, truth, obs, sig = _problem(6, 21)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=7, seed=3, synth_precision=g.SYNTH_FP16)
    r = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    genes = r["genes"].cpu().numpy()
    par = oracle.decode(genes.reshape(-1, 9), si.PRIOR_LO, si.PRIOR_HI)
    stokes = g.me_synth(torch.tensor(par, dtype=torch.float32, device=DEV), lines, grids,
                        fp16=True).cpu().numpy().astype(np.float64)
    L = obs.shape[-1]
    o = obs.cpu().numpy().astype(np.float64)
    s = sig.cpu().numpy().astype(np.float64)
    res = (o[:, None] - stokes.reshape(6, 64, 4, L)) / s[:, None, :, None]
    chi2 = (res ** 2).sum(axis=(2, 3)) / (4 * L - 9)
    fit = r["fitness"].cpu().numpy()
    assert np.allclose(fit, chi2, rtol=1e-3, atol=0)
    # elitism and the reported best
    e = np.argmin(fit, axis=1)
    assert np.array_equal(r["chi2"].cpu().numpy(), fit[np.arange(6), e])
    # against the FP64 forward model: |d chi2| <= (1/nu) sum w^2 (2 |r| delta + delta^2)
    ref = oracle.chi2(par.reshape(6, 64, 9), o, s, olines)
    models = oracle.me_synth(par, olines).reshape(6, 64, 4, L)
    ic = (par[:, 7] + par[:, 8]).reshape(6, 64, 1, 1)
    delta = TOL_MAX * ic
    rr = np.abs(o[:, None] - models)
    w2 = 1.0 / s[:, None, :, None] ** 2
    bound = (w2 * (2 * rr * delta + delta ** 2)).sum(axis=(2, 3)) / (4 * L - 9)
    assert np.all(np.abs(fit - ref) <= bound + 1e-5 * ref)


def test_fp16_loop_is_deterministic_and_splits():
    lines, grids, olines, truth, obs, sig = _problem(9, 22)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=96, generations=6, seed=5, synth_precision=g.SYNTH_FP16)
    r1 = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    r2 = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    assert torch.equal(r1["genes"], r2["genes"]) and torch.equal(r1["fitness"], r2["fitness"])
    cfg2 = g.GAConfig(**{**cfg.__dict__, "pixel_base": 4})
    r3 = g.ga_invert(obs[4:].contiguous(), sig[4:].contiguous(), lines, grids, b, cfg2,
                     want_population=True)
    assert torch.equal(r3["genes"], r1["genes"][4:])


def test_fp16_search_then_fp64_refine_recovers_the_truth():
    # noise-free observations: FP16 synthesis finds the basin, the FP64
    # refinement removes its bias, as with the FP32 search
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(64, 23)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    o32 = torch.tensor(obs.astype(np.float32), device=DEV)
    s32 = torch.tensor(sig.astype(np.float32), device=DEV)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    out = {}
    for name, sp in (("fp32", g.SYNTH_NATIVE), ("fp16", g.SYNTH_FP16)):
        cfg = g.GAConfig(pop=128, generations=150, seed=1, synth_precision=sp)
        r = g.ga_invert(o32, s32, lines, grids, b, cfg)
        ref = g.me_refine_f64(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV),
                              lines, grids, b, r["params"].double().contiguous(), 50)
        out[name] = np.abs(ref["params"][:, 0].cpu().numpy() - truth[:, 0])
    assert np.median(out["fp16"]) <= max(2 * np.median(out["fp32"]), 1.0)
    assert np.percentile(out["fp16"], 75) <= max(2 * np.percentile(out["fp32"], 75), 5.0)
