"""Heuristic first guesses on the GPU (me_first_guess, FP64 per pixel) against
the FP64 oracle, and as seeds of the genetic algorithm.

Both sides evaluate the same formulas in FP64 with different summation
orders (relative 1e-13 in the sums); the outputs are float32, so they agree
to float32 rounding except where a count at half depth sits exactly on the
threshold (one sample moves the half-depth width by a step)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import firstguess as fg
import synth_inputs as si
from conftest import gpu_available

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


@pytest.mark.parametrize("kind", ["slit", "tiny"])
def test_first_guess_matches_oracle(kind):
    lines, grids, olines = _setup(kind)
    truth = si.draw_truth(300, 31)
    mu = np.linspace(0.3, 1.0, 300)
    obs = oracle.me_synth(truth, olines, mu=mu)
    sig = si.sigma_for(truth, mu=mu)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 31)
    got = g.me_first_guess(torch.tensor(obs, device=DEV), grids=grids, lines=lines,
                           bnds=g.bounds(LO, HI),
                           mu=torch.tensor(mu, device=DEV)).cpu().numpy().astype(np.float64)
    ref = fg.first_guess(obs, olines, LO, HI, mu=mu)
    close = np.abs(got - ref) <= 1e-6 * (HI - LO) + 2e-7 * np.abs(ref)
    rows = close.all(axis=1)
    assert rows.mean() >= 0.97, rows.mean()
    # the rest differ only through the half-depth count (Doppler width)
    assert np.all(close[:, [0, 1, 2, 3, 5, 6, 7, 8]])


def test_masked_physics_seeds_enter_the_population():
    # seeds for the parameters the heuristics estimate (B, inclination,
    # v_los), NaN for the rest: seeded slots carry the guesses for those genes
    # only, bit-exact with the oracle's initial population
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(16, 32)
    obs = oracle.me_synth(truth, olines)
    b = g.bounds(LO, HI)
    guess = g.me_first_guess(torch.tensor(obs, device=DEV), lines, grids, b)
    guess[:, [2, 4, 5, 6, 7, 8]] = float("nan")
    for mode in (0, 1):
        cfg = g.GAConfig(pop=64, seed=5, n_seeded=16, seed_jitter=300, seed_params=guess,
                         init_mode=mode)
        got = g.ga_init(16, cfg, b).cpu().numpy()
        gp = guess.cpu().numpy().astype(np.float64)
        for p in range(16):
            ref = oracle.ga_init(5, p, 64, 16, 300, gp[p], LO, HI, init_mode=mode)
            assert np.array_equal(got[p], ref), (mode, p)


@pytest.mark.parametrize("kind", ["slit", "tiny"])
def test_four_seeds_match_oracle(kind):
    """me_seeds against oracle.firstguess.seeds: the same FP64 formulas with
    different summation orders, output as float32.  The field seeds divide
    sums of products whose relative rounding is ~1e-13, so they agree to
    float32 rounding except where an argmin of I or the half-depth count is a
    tie between samples; the polarity box is honoured identically."""
    lines, grids, olines = _setup(kind)
    n = 300
    truth = si.draw_truth(n, 33)
    mu = np.linspace(0.3, 1.0, n)
    obs = oracle.me_synth(truth, olines, mu=mu)
    sig = si.sigma_for(truth, mu=mu)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 33)
    box = np.stack([np.tile(LO, (n, 1)), np.tile(HI, (n, 1))], axis=1).astype(np.float32)
    box[::3, 1, 1] = 90.0                    # polarity restrictions on a third of the pixels
    box[1::3, 0, 1] = 90.0
    b = g.bounds(LO, HI)
    for pb in (None, box):
        got = g.me_seeds(torch.tensor(obs, device=DEV), lines, grids, b,
                         mu=torch.tensor(mu, device=DEV),
                         pixel_bounds=None if pb is None else torch.tensor(pb, device=DEV))
        got = got.cpu().numpy().astype(np.float64)
        ref = fg.seeds(obs, olines, LO, HI, mu=mu,
                       box=None if pb is None else pb.astype(np.float64))
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        fin = ~np.isnan(ref)
        tol = 1e-6 * (HI - LO) + 2e-7 * np.abs(np.nan_to_num(ref))
        close = np.where(fin, np.abs(np.nan_to_num(got) - np.nan_to_num(ref)) <= tol, True)
        rows = close.all(axis=(1, 2))
        print("pixels whose four seeds agree to float rounding: %.3f" % rows.mean())
        assert rows.mean() >= 0.97
        # away from the Doppler width (half-depth count) every seed agrees
        assert close[:, :, [0, 1, 2, 3, 5, 6, 7, 8]].mean() >= 0.995
        if pb is not None:
            inc = got[:, :3, 1]
            assert np.all(inc >= pb[:, 0, 1, None] - 1e-4) and np.all(inc <= pb[:, 1, 1, None] + 1e-4)


def test_seed_sets_enter_the_population_bit_exact():
    """Four guesses per pixel (seed_sets = 4): individual i < n_seeded encodes
    guess i mod 4, exactly for i < 4; bit-exact with the oracle's generation 0."""
    lines, grids, olines = _setup("slit")
    truth = si.draw_truth(12, 34)
    obs = oracle.me_synth(truth, olines)
    b = g.bounds(LO, HI)
    seeds = g.me_seeds(torch.tensor(obs, device=DEV), lines, grids, b)
    for mode, nseed, jit in ((0, 16, 300), (1, 4, 0), (0, 37, 9)):
        cfg = g.GAConfig(pop=64, seed=5, n_seeded=nseed, seed_jitter=jit, seed_params=seeds,
                         init_mode=mode, pixel_base=40)
        got = g.ga_init(12, cfg, b).cpu().numpy()
        sp = seeds.cpu().numpy().astype(np.float64)
        for p in range(12):
            ref = oracle.ga_init(5, 40 + p, 64, nseed, jit, sp[p], LO, HI, init_mode=mode)
            assert np.array_equal(got[p], ref), (mode, p)
        # the first four individuals decode to the four seeds' codes
        gi = got[:, :4].astype(np.int64)
        exact = np.floor(np.clip((sp - LO) / (HI - LO), 0, 1) * 65535 + 0.5)
        seeded = ~np.isnan(sp)
        assert np.array_equal(gi[seeded], exact[seeded])


def test_seeded_inversion_matches_oracle_trajectory_fp64():
    """The FP64 loop seeded with the four seeds follows the oracle's
    trajectory (same integer steps, fitness to FP64 rounding)."""
    lines, grids, olines = _setup("tiny")
    truth = si.draw_truth(6, 35)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 35)
    b = g.bounds(LO, HI)
    seeds = g.me_seeds(torch.tensor(obs, device=DEV), lines, grids, b)
    cfg = g.GAConfig(pop=32, generations=12, seed=2, n_seeded=8, seed_jitter=200,
                     seed_params=seeds)
    res = g.ga_invert(torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), lines, grids,
                      b, cfg, want_population=True)
    ref = oracle.ga_invert(obs, sig, olines, LO, HI, pop=32, generations=12, k=4, p_cross=0.85,
                           p_mut=0.05, seed=2, n_seeded=8, seed_jitter=200,
                           seed_params=seeds.cpu().numpy().astype(np.float64),
                           want_population=True)
    same = [np.array_equal(res["genes"][p].cpu().numpy(), ref["genes"][p]) for p in range(6)]
    assert sum(same) >= 5, same
