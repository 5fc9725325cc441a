"""Non-magnetic pre-fit (Sec. 5.3), per-pixel search boxes (Sec. 5.3 ranges,
Sec. 5.5 polarity) and the genetic algorithm inside per-pixel boxes, through
the C ABI, against the oracle.

Bars: the pre-fit as the refinement it reuses (same minimum as the oracle's
for at least 9 of 10 pixels, chi-square to 1e-7); the boxes bit-exact against
the oracle's rounded to float (the polarity decision compares a sum with a
threshold, and the sums differ only in order: a pixel within 1e-9 of the
threshold would be ambiguous, which these seeded inputs do not contain); the
genetic algorithm in per-pixel boxes bit-exact against the same pixels run
alone with their boxes as the common box (FP32, FP16 synthesis and the
service), and on the oracle's trajectory in FP64."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from conftest import gpu_available
from oracle import firstguess as ofg
from oracle import searchbox as osb

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


def _t(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


def _noisy(olines, n, seed):
    truth = si.draw_truth(n, seed)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    return truth, obs + sig[:, :, None] * si.std_normal(obs.shape, seed), sig


def test_prefit_matches_oracle():
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 10, 21)
    start = ofg.first_guess(obs, olines, LO, HI)
    r = g.me_prefit_f64(_t(obs), _t(sig), lines, grids, g.bounds(LO, HI), _t(start), 30)
    ref = oracle.prefit(obs, sig, olines, LO, HI, start, 30)
    gp = r["params"].cpu().numpy()
    assert np.all(gp[:, 0] == 0.0)
    dx = np.abs(gp - ref["params"]) / (HI - LO)
    same = dx.max(axis=1) < 1e-6
    print("pixels at the oracle's minimum: %d / 10" % same.sum())
    assert same.sum() >= 9
    gc, rc = r["chi2"].cpu().numpy(), ref["chi2"]
    assert np.all(np.abs(gc[same] - rc[same]) <= 1e-7 * rc[same])


def test_prefit_rejects_a_box_without_zero_field():
    lines, grids, olines = _setup("tiny")
    lo = LO.copy()
    lo[0] = 50.0
    z = torch.zeros((1, 4, sum(gr.n for gr in grids)), dtype=torch.float64, device=DEV)
    with pytest.raises(g.GenesisError):
        g.me_prefit_f64(z, torch.ones((1, 4), dtype=torch.float64, device=DEV), lines, grids,
                        g.bounds(lo, HI), torch.zeros((1, 9), dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("with_prefit", [False, True])
def test_search_box_matches_oracle(with_prefit):
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 96, 22)
    pf = None
    if with_prefit:
        pf = oracle.prefit(obs, sig, olines, LO, HI, ofg.first_guess(obs, olines, LO, HI),
                           10)["params"]
    box = g.me_search_box(_t(obs), _t(sig), lines, grids, g.bounds(LO, HI),
                          prefit=None if pf is None else _t(pf), polarity_nsigma=3.0)
    ref = osb.search_box(obs, sig, olines, LO, HI, prefit=pf, n_sigma=3.0).astype(np.float32)
    assert np.array_equal(box.cpu().numpy(), ref)
    # the restriction is used: strong-field pixels get one polarity
    restricted = (ref[:, 1, 1] - ref[:, 0, 1]) == 90.0
    assert restricted.sum() >= 20


def _boxes(n, seed):
    rng = np.random.default_rng(seed)
    a = LO + (HI - LO) * rng.uniform(0, 0.5, (n, 9))
    b = a + (HI - LO) * rng.uniform(0.2, 0.5, (n, 9))
    return np.stack([a, np.minimum(b, HI)], axis=1).astype(np.float32)


@pytest.mark.parametrize("synth", [0, 1])
def test_pixel_boxes_equal_single_pixel_runs(synth):
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 6, 23)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    box = _boxes(6, 24)
    kw = dict(pop=64, generations=12, seed=5, synth_precision=synth, init_mode=1,
              restart_every=5)
    cfg = g.GAConfig(pixel_bounds=_t(box, torch.float32), **kw)
    r = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg, want_population=True)
    assert torch.all(r["status"] == 0)
    for p in range(6):
        alone = g.ga_invert(o32[p:p + 1].contiguous(), s32[p:p + 1].contiguous(), lines, grids,
                            g.bounds(box[p, 0].astype(np.float64), box[p, 1].astype(np.float64)),
                            g.GAConfig(pixel_base=p, **kw), want_population=True)
        assert torch.equal(r["genes"][p], alone["genes"][0]), p
        assert torch.equal(r["params"][p], alone["params"][0]), p
        assert torch.equal(r["chi2"][p], alone["chi2"][0]), p


def test_common_box_per_pixel_changes_nothing():
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 5, 25)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    lo32, hi32 = LO.astype(np.float32), HI.astype(np.float32)
    b = g.bounds(lo32.astype(np.float64), hi32.astype(np.float64))
    common = np.stack([np.broadcast_to(lo32, (5, 9)), np.broadcast_to(hi32, (5, 9))], axis=1)
    cfg = g.GAConfig(pop=64, generations=8, seed=2)
    a = g.ga_invert(o32, s32, lines, grids, b, cfg, want_population=True)
    cfg.pixel_bounds = _t(common, torch.float32)
    c = g.ga_invert(o32, s32, lines, grids, b, cfg, want_population=True)
    assert torch.equal(a["genes"], c["genes"]) and torch.equal(a["params"], c["params"])


def test_f64_pixel_boxes_track_the_oracle():
    lines, grids, olines = _setup("tiny")
    truth, obs, sig = _noisy(olines, 12, 26)
    box = _boxes(12, 27).astype(np.float64)
    cfg = g.GAConfig(pop=48, generations=10, tournament_k=4, seed=3,
                     pixel_bounds=_t(box.astype(np.float32), torch.float32))
    r = g.ga_invert(_t(obs), _t(sig), lines, grids, g.bounds(LO, HI), cfg, want_population=True)
    ref = oracle.ga_invert(obs, sig, olines, LO, HI, pop=48, generations=10, k=4,
                           p_cross=cfg.p_cross, p_mut=cfg.p_mut, seed=3, want_population=True,
                           pixel_box=box.astype(np.float32).astype(np.float64))
    same = [np.array_equal(r["genes"][p].cpu().numpy(), ref["genes"][p]) for p in range(12)]
    # bit-exact operators; a fitness near-tie (1e-13 relative) may flip a decision
    assert sum(same) >= 10, same
    c, cr = r["chi2"].cpu().numpy(), ref["chi2"]
    assert np.all(np.abs(c - cr)[same] <= 1e-9 * cr[same])


def test_invalid_pixel_boxes_give_status_3():
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 4, 28)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    box = _boxes(4, 29)
    box[1, 1, 4] = box[1, 0, 4] - 1e-3     # hi < lo
    box[2, 0, 0] = np.nan
    box[3, 1, 5] = 1.2                      # damping above 1: fine in FP32, not for FP16
    cfg = g.GAConfig(pop=32, generations=3, seed=1, pixel_bounds=_t(box, torch.float32))
    r = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg)
    assert r["status"].cpu().tolist() == [0, 3, 3, 0]
    p = r["params"].cpu().numpy()
    assert np.all(np.isnan(p[1:3])) and np.isfinite(p[[0, 3]]).all()
    cfg.synth_precision = g.SYNTH_FP16
    r16 = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg)
    assert r16["status"].cpu().tolist() == [0, 3, 3, 3]


def test_seeded_init_in_pixel_boxes_matches_oracle():
    npix, pop = 5, 40
    box = _boxes(npix, 30)
    seeds = si.draw_uniform_box(npix, 31).astype(np.float32)
    cfg = g.GAConfig(pop=pop, tournament_k=4, seed=11, n_seeded=6, seed_jitter=300,
                     seed_params=_t(seeds, torch.float32), pixel_bounds=_t(box, torch.float32))
    got = g.ga_init(npix, cfg, g.bounds(LO, HI)).cpu().numpy()
    for p in range(npix):
        ref = oracle.ga_init(11, p, pop, 6, 300, seeds[p].astype(np.float64),
                             box[p, 0].astype(np.float64), box[p, 1].astype(np.float64))
        assert np.array_equal(got[p], ref), p


def test_serving_with_pixel_boxes_equals_ga_invert():
    lines, grids, olines = _setup("slit")
    truth, obs, sig = _noisy(olines, 30, 32)
    o32, s32 = _t(obs, torch.float32), _t(sig, torch.float32)
    box = osb.search_box(obs, sig, olines, LO, HI, n_sigma=3.0).astype(np.float32)
    cfg = g.GAConfig(pop=64, generations=15, seed=4, pixel_bounds=_t(box, torch.float32))
    alone = g.ga_invert(o32, s32, lines, grids, g.bounds(LO, HI), cfg)
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=4)
    rid = sess.submit(o32, s32, lines, grids, g.bounds(LO, HI), cfg)
    for _ in range(20):
        if sess.poll(rid):
            break
        sess.step()
        torch.cuda.synchronize()
    out = sess.result(rid)
    assert torch.equal(out["params"], alone["params"])
    assert torch.equal(out["chi2"], alone["chi2"])
    sess.close()
