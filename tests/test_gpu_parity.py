"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Forward model: FP32 within 1e-5 of the continuum intensity Ic = S0 + mu S1 at
every sample (the FP32 rational Voigt approximation is good to 1.5e-7, which moves
the Stokes vector by at most 2.8e-6 Ic over random models including eta0 = 30, and its
FP32 evaluation to ~4e-7, which moves profiles by < 1e-6 Ic), FP64 within
1e-10 Ic: the oracle forms lambda_j - lambda_c from absolute wavelengths near
6302 A, whose FP64 rounding (ulp 9e-13 A) over the narrowest Doppler width
(0.02 A) moves v by 4.5e-11, and |dI/dv| <= 0.92 mu S1.  Integer genetic
operators: bit-exact.  The whole inversion: the
fused single-launch loop equals the step-by-step composition of the library's
own operator entry points bit for bit, and every number it reports agrees with
the oracle re-evaluated on it.
"""
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
FWD_TOL_F32 = 1e-5
FWD_TOL_F64 = 1e-10


def _setup(kind, nlam=None):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set(kind):
        n = nlam or n
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       start, step, n))
    return lines, grids, olines


def _params(n, seed):
    """Uniform box draws plus the degenerate corners of the model."""
    p = si.draw_uniform_box(n, seed)
    k = n // 10
    p[:k, 0] = 0.0                      # zero field
    p[k:2 * k, 1] = 0.0                 # longitudinal
    p[2 * k:3 * k, 1] = 90.0            # transverse
    p[3 * k:4 * k, 1] = 180.0
    p[4 * k:5 * k, 5] = 0.0             # pure Gaussian core (a = 0)
    p[5 * k:6 * k, 6] = 30.0            # saturated line
    p[6 * k:7 * k, 7] = 0.0             # S0 = 0
    p[7 * k:8 * k, 0] = 3000.0          # strongest field
    p[7 * k:8 * k, 4] = 0.02            # narrowest line
    return p


def _ic(p, mu=None):
    m = 1.0 if mu is None else mu
    return p[:, 7] + m * p[:, 8]


# --------------------------------------------------------------------------- #
# forward model

@pytest.mark.parametrize("kind", ["tiny", "slit"])
@pytest.mark.parametrize("n", [1, 637])
def test_me_synth_f32_parity(kind, n):
    lines, grids, olines = _setup(kind)
    p = _params(n, seed=n + len(kind))
    p32 = p.astype(np.float32)
    ref = oracle.me_synth(p32.astype(np.float64), olines)
    got = g.me_synth(torch.tensor(p32, device=DEV), lines, grids).cpu().numpy()
    err = np.max(np.abs(got - ref), axis=(1, 2)) / _ic(p32.astype(np.float64))
    print("f32 max err / Ic = %.3e (median %.3e)" % (err.max(), np.median(err)))
    assert err.max() < FWD_TOL_F32


@pytest.mark.parametrize("kind", ["tiny", "slit"])
def test_me_synth_f64_parity(kind):
    lines, grids, olines = _setup(kind)
    p = _params(300, seed=3)
    mu = np.random.default_rng(1).uniform(0.1, 1.0, len(p))
    ref = oracle.me_synth(p, olines, mu)
    got = g.me_synth(torch.tensor(p, device=DEV), lines, grids,
                     mu=torch.tensor(mu, device=DEV)).cpu().numpy()
    err = np.max(np.abs(got - ref), axis=(1, 2)) / _ic(p, mu)
    print("f64 max err / Ic = %.3e" % err.max())
    assert err.max() < FWD_TOL_F64


def test_me_synth_mu_and_empty():
    lines, grids, olines = _setup("tiny")
    p = _params(70, seed=5).astype(np.float32)
    mu = np.random.default_rng(2).uniform(0.05, 1.0, len(p)).astype(np.float32)
    ref = oracle.me_synth(p.astype(np.float64), olines, mu.astype(np.float64))
    got = g.me_synth(torch.tensor(p, device=DEV), lines, grids,
                     mu=torch.tensor(mu, device=DEV)).cpu().numpy()
    assert np.max(np.abs(got - ref), axis=(1, 2)).max() < FWD_TOL_F32
    empty = g.me_synth(torch.empty((0, 9), device=DEV), lines, grids)
    assert empty.shape == (0, 4, 100)


def _chi2_tol(obs, ref_model, sig, ic, nu, delta_rel):
    """|chi2_gpu - chi2_ref| bound from a forward-model error delta = delta_rel Ic
    at every sample: (1/nu) sum w^2 (2 |r| delta + delta^2), plus FP32
    accumulation error."""
    r = np.abs(obs[:, None] - ref_model)
    w2 = 1.0 / sig[:, None, :, None] ** 2
    d = delta_rel * ic[:, None, None, None]
    return (w2 * (2 * r * d + d * d)).sum(axis=(2, 3)) / nu


@pytest.mark.parametrize("kind", ["tiny", "slit"])
def test_me_chi2_parity(kind):
    lines, grids, olines = _setup(kind)
    npix, pop = 5, 70
    truth = si.draw_truth(npix, seed=11)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 3)
    obs32, sig32 = obs.astype(np.float32), sig.astype(np.float32)
    par = np.stack([_params(pop, seed=20 + i) for i in range(npix)]).astype(np.float32)
    par[:, 0] = truth                   # include the truth itself
    par[:, 0] = par[:, 0].astype(np.float32)
    ref = oracle.chi2(par.astype(np.float64), obs32.astype(np.float64),
                      sig32.astype(np.float64), olines)
    got = g.me_chi2(torch.tensor(par, device=DEV), torch.tensor(obs32, device=DEV),
                    torch.tensor(sig32, device=DEV), lines, grids).cpu().numpy()
    L = obs.shape[-1]
    models = oracle.me_synth(par.reshape(-1, 9).astype(np.float64), olines).reshape(npix, pop, 4, L)
    tol = _chi2_tol(obs32.astype(np.float64), models, sig32.astype(np.float64),
                    _ic(truth), 4 * L - 9, FWD_TOL_F32) + 1e-5 * ref
    assert np.all(np.abs(got - ref) <= tol)
    # f64
    got64 = g.me_chi2(torch.tensor(par.astype(np.float64), device=DEV),
                      torch.tensor(obs32.astype(np.float64), device=DEV),
                      torch.tensor(sig32.astype(np.float64), device=DEV),
                      lines, grids).cpu().numpy()
    assert np.max(np.abs(got64 - ref) / np.maximum(ref, 1e-3)) < 1e-9


def test_chi2_bad_pixels_are_nan():
    lines, grids, olines = _setup("tiny")
    truth = si.draw_truth(3, seed=1)
    obs = oracle.me_synth(truth, olines).astype(np.float32)
    sig = si.sigma_for(truth).astype(np.float32)
    obs[1, 0, 3] = np.inf
    sig[2, 1] = -1.0
    par = np.repeat(truth[:, None, :], 4, axis=1).astype(np.float32)
    got = g.me_chi2(torch.tensor(par, device=DEV), torch.tensor(obs, device=DEV),
                    torch.tensor(sig, device=DEV), lines, grids).cpu().numpy()
    assert np.isfinite(got[0]).all() and np.isnan(got[1:]).all()


# --------------------------------------------------------------------------- #
# integer operators: bit-exact

def test_ga_init_bit_exact():
    cfg = g.GAConfig(pop=70, seed=(123 << 32) | 99, pixel_base=1000)
    got = g.ga_init(5, cfg).cpu().numpy()
    for p in range(5):
        assert np.array_equal(got[p], oracle.ga_init(cfg.seed, 1000 + p, 70))


def test_ga_decode_exact():
    genes = si.random_genes(3, 50, 4)
    genes[0, 0] = 0
    genes[0, 1] = 65535
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    got = g.ga_decode(torch.tensor(genes, device=DEV), b).cpu().numpy()
    ref = oracle.decode(genes.reshape(-1, 9), si.PRIOR_LO, si.PRIOR_HI).reshape(genes.shape)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("pop,k,pc,pm", [(64, 4, 0.85, 0.05), (128, 4, 0.85, 0.05),
                                         (70, 1, 0.0, 0.3), (33, 8, 1.0, 0.0),
                                         (2, 2, 0.5, 0.05), (200, 3, 0.85, 1.0),
                                         (1024, 8, 0.85, 0.05)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_ga_step_bit_exact(pop, k, pc, pm, dtype):
    npix = 6
    genes = si.random_genes(npix, pop, pop + k)
    fit = si.random_fitness(npix, pop, pop * k, ties=True, nans=(pop >= 16))
    fit = fit.astype(np.float32).astype(np.float64)       # exactly representable in both
    cfg = g.GAConfig(pop=pop, tournament_k=k, p_cross=pc, p_mut=pm, seed=77, pixel_base=5)
    gen = 3
    res = g.ga_step(torch.tensor(genes, device=DEV), torch.tensor(fit, dtype=dtype, device=DEV),
                    cfg, gen)
    res = {kk: v.cpu().numpy() for kk, v in res.items()}
    pc32 = float(np.float32(pc))
    pm32 = float(np.float32(pm))
    for p in range(npix):
        ref = oracle.ga_step(genes[p], fit[p], k, pc32, pm32, 77, 5 + p, gen)
        assert np.array_equal(res["genes"][p], ref["genes"])
        assert np.array_equal(res["parents"][p], ref["parents"])
        assert np.array_equal(res["xpoint"][p], ref["xpoint"])
        assert np.array_equal(res["masks"][p], ref["masks"])
        assert res["elite"][p] == ref["elite"]


# --------------------------------------------------------------------------- #
# the whole loop

def _problem(kind, npix, seed, noise=True, dtype=np.float32):
    lines, grids, olines = _setup(kind)
    truth = si.draw_truth(npix, seed)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    if noise:
        obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return lines, grids, olines, truth, obs.astype(dtype), sig.astype(dtype)


def _stepwise(obs_t, sig_t, lines, grids, b, cfg):
    genes = g.ga_init(obs_t.shape[0], cfg, b)
    fit = g.ga_evaluate(genes, b, obs_t, sig_t, lines, grids)
    for t in range(1, cfg.generations + 1):
        genes = g.ga_step(genes, fit, cfg, t, diagnostics=False)["genes"]
        fit = g.ga_evaluate(genes, b, obs_t, sig_t, lines, grids)
    return genes, fit


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("pop", [64, 96])
def test_fused_loop_equals_stepwise_composition(dtype, pop):
    lines, grids, olines, truth, obs, sig = _problem("slit", 7, 4, dtype=dtype)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=pop, generations=6, tournament_k=4, seed=9, pixel_base=3)
    obs_t, sig_t = torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV)
    fused = g.ga_invert(obs_t, sig_t, lines, grids, b, cfg, want_population=True)
    genes, fit = _stepwise(obs_t, sig_t, lines, grids, b, cfg)
    assert torch.equal(fused["genes"], genes)
    assert torch.equal(fused["fitness"], fit)
    # best = argmin of the last generation, decoded
    f = fit.cpu().numpy()
    e = np.argmin(np.where(np.isnan(f), np.inf, f), axis=1)
    assert np.array_equal(fused["chi2"].cpu().numpy(), f[np.arange(len(e)), e])
    gb = genes.cpu().numpy()[np.arange(len(e)), e]
    dec = oracle.decode(gb, si.PRIOR_LO, si.PRIOR_HI).astype(dtype)
    assert np.array_equal(fused["params"].cpu().numpy(), dec)


def test_fused_loop_at_the_largest_population():
    # GENESIS_MAX_POP = 1024 lanes: sixteen waves per workgroup
    lines, grids, olines, truth, obs, sig = _problem("slit", 3, 14)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=1024, generations=3, tournament_k=8, seed=4, init_mode=1,
                     restart_every=2)
    obs_t, sig_t = torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV)
    fused = g.ga_invert(obs_t, sig_t, lines, grids, b, cfg, want_population=True)
    genes = g.ga_init(3, cfg, b)
    fit = g.ga_evaluate(genes, b, obs_t, sig_t, lines, grids)
    for t in range(1, cfg.generations + 1):
        if t - 1 > 0 and (t - 1) % cfg.restart_every == 0:
            genes = g.ga_restart(genes, fit, cfg, t - 1)
            fit = g.ga_evaluate(genes, b, obs_t, sig_t, lines, grids)
        genes = g.ga_step(genes, fit, cfg, t, diagnostics=False)["genes"]
        fit = g.ga_evaluate(genes, b, obs_t, sig_t, lines, grids)
    assert torch.equal(fused["genes"], genes)
    assert torch.equal(fused["fitness"], fit)


def test_long_ragged_lines():
    # 2 x 1001 samples (L = 2002, not a multiple of the 64-lane waves): the
    # staged observation fills 32 KB of LDS; the loop equals its composition
    # and its fitness is the oracle's chi-square of the decoded genes
    lines, grids, olines = [], [], []
    for ln in (si.FE6301, si.FE6302):
        st, sp = si.grid(ln, 1001, half_width=0.6)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, 1001))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, 1001))
    truth = si.draw_truth(3, 15)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = (obs + sig[:, :, None] * si.std_normal(obs.shape, 15)).astype(np.float32)
    sig = sig.astype(np.float32)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=2, seed=6)
    obs_t, sig_t = torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV)
    fused = g.ga_invert(obs_t, sig_t, lines, grids, b, cfg, want_population=True)
    genes, fit = _stepwise(obs_t, sig_t, lines, grids, b, cfg)
    assert torch.equal(fused["genes"], genes) and torch.equal(fused["fitness"], fit)
    par = oracle.decode(genes.cpu().numpy().reshape(-1, 9), si.PRIOR_LO,
                        si.PRIOR_HI).reshape(3, 64, 9)
    o64, s64 = obs.astype(np.float64), sig.astype(np.float64)
    ref = oracle.chi2(par, o64, s64, olines)
    L = obs.shape[-1]
    models = oracle.me_synth(par.reshape(-1, 9), olines).reshape(3, 64, 4, L)
    # FP32 accumulation over 2002 samples per Stokes parameter: 8x the slit row's allowance
    tol = _chi2_tol(o64, models, s64, _ic(truth), 4 * L - 9, FWD_TOL_F32) + 8e-5 * ref
    assert np.all(np.abs(fit.cpu().numpy() - ref) <= tol)


def test_fitness_matches_oracle_on_decoded_genes():
    lines, grids, olines, truth, obs, sig = _problem("slit", 3, 8)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=3, seed=2)
    res = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                      b, cfg, want_population=True)
    genes = res["genes"].cpu().numpy()
    par = oracle.decode(genes.reshape(-1, 9), si.PRIOR_LO, si.PRIOR_HI).reshape(genes.shape)
    o64, s64 = obs.astype(np.float64), sig.astype(np.float64)
    ref = oracle.chi2(par, o64, s64, olines)
    L = obs.shape[-1]
    models = oracle.me_synth(par.reshape(-1, 9), olines).reshape(par.shape[0], par.shape[1], 4, L)
    tol = _chi2_tol(o64, models, s64, _ic(truth), 4 * L - 9, FWD_TOL_F32) + 1e-5 * ref
    assert np.all(np.abs(res["fitness"].cpu().numpy() - ref) <= tol)


def test_loop_determinism_pixel_base_and_status():
    lines, grids, olines, truth, obs, sig = _problem("tiny", 9, 5)
    obs[4, 2, 7] = np.nan
    sig[6, 0] = 0.0
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=8, seed=5)
    o, s = torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV)
    r1 = g.ga_invert(o, s, lines, grids, b, cfg, want_population=True)
    r2 = g.ga_invert(o, s, lines, grids, b, cfg, want_population=True)
    for k in ("genes", "status"):
        assert torch.equal(r1[k], r2[k])
    assert torch.equal(r1["chi2"].nan_to_num(-1), r2["chi2"].nan_to_num(-1))
    st = r1["status"].cpu().numpy()
    assert st[4] == 1 and st[6] == 2 and (np.delete(st, [4, 6]) == 0).all()
    c = r1["chi2"].cpu().numpy()
    assert np.isnan(c[[4, 6]]).all() and np.isfinite(np.delete(c, [4, 6])).all()
    # splitting the map with pixel_base reproduces the single call
    cfg2 = g.GAConfig(pop=64, generations=8, seed=5, pixel_base=5)
    r3 = g.ga_invert(o[5:].contiguous(), s[5:].contiguous(), lines, grids, b, cfg2,
                     want_population=True)
    assert torch.equal(r3["genes"], r1["genes"][5:])
    # empty input
    r0 = g.ga_invert(o[:0], s[:0], lines, grids, b, cfg)
    assert r0["params"].shape == (0, 9)


def test_issue_priority_leaves_results_unchanged():
    # A launch with more pixels than the device holds at once (16,384 one-wave
    # workgroups against 256 CUs x 16) keeps the default issue priority; one
    # that fits (256 pixels) sets it every generation from the workgroup's
    # lag behind its XCD's average progress.  Priority orders instruction
    # issue only, so every pixel's result is the same either way.
    lines, grids, _ = _setup("tiny")
    npix = 16384
    truth = si.draw_truth(npix, 31)
    obs = g.me_synth(torch.tensor(truth, dtype=torch.float32, device=DEV), lines, grids)
    sig = torch.tensor(si.sigma_for(truth), dtype=torch.float32, device=DEV)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=3, seed=7)
    big = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    part = g.ga_invert(obs[:256].contiguous(), sig[:256].contiguous(), lines, grids, b, cfg,
                       want_population=True)
    for k in ("genes", "params", "chi2", "status"):
        assert torch.equal(part[k], big[k][:256]), k


def test_overlapping_single_round_launches_share_the_progress_counter_harmlessly():
    # Two single-round launches queued on two streams may run at the same
    # time and then share the device's progress counters: only the issue
    # order changes, so each result equals the same launch run alone.
    lines, grids, _ = _setup("tiny")
    truth = si.draw_truth(512, 33)
    obs = g.me_synth(torch.tensor(truth, dtype=torch.float32, device=DEV), lines, grids)
    sig = torch.tensor(si.sigma_for(truth), dtype=torch.float32, device=DEV)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    halves = [(obs[:256].contiguous(), sig[:256].contiguous(),
               g.GAConfig(pop=64, generations=40, seed=5)),
              (obs[256:].contiguous(), sig[256:].contiguous(),
               g.GAConfig(pop=64, generations=25, seed=6))]
    alone = [g.ga_invert(o, s_, lines, grids, b, c, want_population=True) for o, s_, c in halves]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    both = []
    for st, (o, s_, c) in zip(streams, halves):
        with torch.cuda.stream(st):
            both.append(g.ga_invert(o, s_, lines, grids, b, c, want_population=True))
    torch.cuda.synchronize()
    for a, r in zip(alone, both):
        for k in ("genes", "params", "chi2", "status"):
            assert torch.equal(a[k], r[k]), k


def test_loop_generation_zero_is_the_initial_population():
    lines, grids, olines, truth, obs, sig = _problem("tiny", 3, 6)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=65, generations=0, seed=12)
    r = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                    b, cfg, want_population=True)
    for p in range(3):
        assert np.array_equal(r["genes"][p].cpu().numpy(), oracle.ga_init(12, p, 65))


def test_f64_loop_tracks_the_oracle():
    """FP64 fused loop vs the oracle's loop on the small single-line workload:
    the operators are bit-exact, so trajectories agree while fitness values
    agree to the ordering of every tournament; near-ties (1e-13 relative) may
    flip a decision, after which the two runs are different but equally valid
    samples of the heuristic.  Require most pixels to agree exactly and all to
    reach comparable chi-square."""
    lines, grids, olines, truth, obs, sig = _problem("tiny", 16, 0, dtype=np.float64)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=15, tournament_k=4, seed=0)
    r = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                    b, cfg, want_population=True)
    ref = oracle.ga_invert(obs, sig, olines, si.PRIOR_LO, si.PRIOR_HI, pop=64, generations=15,
                           k=4, p_cross=float(np.float32(0.85)), p_mut=float(np.float32(0.05)),
                           seed=0, want_population=True)
    same = [np.array_equal(r["genes"][p].cpu().numpy(), ref["genes"][p]) for p in range(16)]
    print("pixels with identical final populations: %d / 16" % sum(same))
    assert sum(same) >= 12
    # identical genotypes: chi-square within the FP64 forward-model bound
    bp = r["params"].cpu().numpy()
    L = obs.shape[-1]
    models = oracle.me_synth(bp, olines)[:, None]
    tol = _chi2_tol(obs, models, sig, _ic(truth), 4 * L - 9, FWD_TOL_F64)[:, 0]
    for p in np.nonzero(same)[0]:
        assert abs(r["chi2"][p].item() - ref["chi2"][p]) <= tol[p]


@pytest.mark.parametrize("pc,k,pop", [(0.0, 3, 16), (0.0, 8, 8), (1.0, 8, 8)])
def test_f64_loop_special_cases_match_the_oracle(pc, k, pop):
    """The FP64 fused loop in the oracle's exactly pinned regimes (no
    mutation; no crossover, or a tournament over the whole population):
    final populations equal the oracle's, and they hold only generation-0
    genotypes, or only copies of generation 0's best."""
    lines, grids, olines, truth, obs, sig = _problem("tiny", 4, 4, dtype=np.float64)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=pop, generations=6, tournament_k=k, p_cross=pc, p_mut=0.0, seed=5)
    r = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                    b, cfg, want_population=True)
    kw = dict(pop=pop, k=k, p_cross=pc, p_mut=0.0, seed=5, want_population=True)
    ref = oracle.ga_invert(obs, sig, olines, si.PRIOR_LO, si.PRIOR_HI, generations=6, **kw)
    ref0 = oracle.ga_invert(obs, sig, olines, si.PRIOR_LO, si.PRIOR_HI, generations=0, **kw)
    for p in range(4):
        genes = r["genes"][p].cpu().numpy()
        assert np.array_equal(genes, ref["genes"][p])
        first = {tuple(x) for x in ref0["genes"][p].tolist()}
        assert all(tuple(x) in first for x in genes.tolist())
        if k == pop:
            best = ref0["genes"][p][np.argmin(ref0["fitness"][p])]
            assert np.array_equal(genes, np.broadcast_to(best, genes.shape))


def test_tiny_workload_at_full_size_tracks_the_oracle():
    """The single-line FP64 workload at its full size (64 pixels, population
    64, 100 generations, seed 0) against the oracle's loop: every operator is
    bit-exact, so final populations agree wherever no tournament met a
    fitness near-tie on the way; allow a few such pixels and require the
    median chi-square over all pixels to agree."""
    lines, grids, olines, truth, obs, sig = _problem("tiny", 64, 0, dtype=np.float64)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=100, tournament_k=4, seed=0)
    r = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                    b, cfg, want_population=True)
    ref = oracle.ga_invert(obs, sig, olines, si.PRIOR_LO, si.PRIOR_HI, pop=64, generations=100,
                           k=4, p_cross=float(np.float32(0.85)), p_mut=float(np.float32(0.05)),
                           seed=0, want_population=True)
    same = np.array([np.array_equal(r["genes"][p].cpu().numpy(), ref["genes"][p])
                     for p in range(64)])
    c, cr = r["chi2"].cpu().numpy(), ref["chi2"]
    print("identical final populations: %d / 64" % same.sum())
    assert same.sum() >= 56
    bp = r["params"].cpu().numpy()
    models = oracle.me_synth(bp, olines)[:, None]
    tol = _chi2_tol(obs, models, sig, _ic(truth), 4 * obs.shape[-1] - 9, FWD_TOL_F64)[:, 0]
    assert np.all(np.abs(c[same] - cr[same]) <= tol[same])
    assert abs(np.median(c) / np.median(cr) - 1) < 0.02


@pytest.mark.parametrize("kind", ["tiny", "slit"])
def test_loop_reduces_chi2_and_beats_truth_on_noisy_data(kind):
    lines, grids, olines, truth, obs, sig = _problem(kind, 16, 21)
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    o, s = torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV)
    r0 = g.ga_invert(o, s, lines, grids, b, g.GAConfig(pop=128, generations=0, seed=1))
    r = g.ga_invert(o, s, lines, grids, b, g.GAConfig(pop=128, generations=200, seed=1))
    c0, c = r0["chi2"].cpu().numpy(), r["chi2"].cpu().numpy()
    assert np.all(c <= c0)
    assert np.median(c / c0) < 0.02


# --------------------------------------------------------------------------- #
# full-size workload (2048 pixels x 2 lines x 128 samples, pop 128, G 200):
# sampled pixels checked against the oracle one by one

def test_full_size_slit_row_sampled():
    lines, grids, olines = _setup("slit")
    npix = 2048
    truth = si.draw_truth(npix, seed=0)
    p32 = torch.tensor(truth.astype(np.float32), device=DEV)
    obs = g.me_synth(p32, lines, grids)
    sig = torch.tensor(si.sigma_for(truth).astype(np.float32), device=DEV)
    obs = obs + sig[:, :, None] * torch.tensor(si.std_normal(tuple(obs.shape), 0),
                                               dtype=torch.float32, device=DEV)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(npix, 12, replace=False))
    # forward model on sampled pixels
    ref = oracle.me_synth(truth[sample].astype(np.float32).astype(np.float64), olines)
    noise_free = g.me_synth(p32, lines, grids).cpu().numpy()[sample]
    assert (np.max(np.abs(noise_free - ref), axis=(1, 2)) / _ic(truth[sample])).max() < FWD_TOL_F32
    # the inversion as the benchmark runs it
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=128, generations=200, tournament_k=4, p_cross=0.85, p_mut=0.05, seed=0)
    r = g.ga_invert(obs.contiguous(), sig, lines, grids, b, cfg, want_population=True)
    o64 = obs.double().cpu().numpy()[sample]
    s64 = sig.double().cpu().numpy()[sample]
    bp = r["params"].double().cpu().numpy()[sample]
    c_or = oracle.chi2(bp[:, None, :], o64, s64, olines)[:, 0]
    c_gpu = r["chi2"].double().cpu().numpy()[sample]
    L = o64.shape[-1]
    models = oracle.me_synth(bp, olines)[:, None]
    tol = _chi2_tol(o64, models, s64, _ic(truth[sample]), 4 * L - 9, FWD_TOL_F32)[:, 0] + 1e-5 * c_or
    assert np.all(np.abs(c_gpu - c_or) <= tol)
    # elitism: the reported best is the minimum of the final population
    f = r["fitness"].cpu().numpy()
    assert np.array_equal(r["chi2"].cpu().numpy(), np.nanmin(f, axis=1))
    # the best beats the noisy truth's chi-square on most pixels
    c_truth = oracle.chi2(truth[sample][:, None, :], o64, s64, olines)[:, 0]
    print("chi2 best / chi2 truth:", np.round(c_gpu / c_truth, 3))
