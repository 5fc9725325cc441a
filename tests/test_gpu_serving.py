"""Continuous-batching service: every request's result is bit-identical to a
standalone ga_invert of the same request, alone or mixed with others arriving
at different times, and every served number agrees with the FP64 oracle
re-evaluated on it; admission respects the memory budget; cancellation;
released requests leave no memory behind."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from conftest import gpu_available
from tolerances import FWD_TOL_F32, chi2_tol, ic_of, recover_genes

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"


def _request(kind, npix, seed, bad=False):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set(kind):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    truth = si.draw_truth(npix, seed)
    obs = oracle.me_synth(truth, olines)
    sig = si.sigma_for(truth)
    obs = (obs + sig[:, :, None] * si.std_normal(obs.shape, seed)).astype(np.float32)
    sig = sig.astype(np.float32)
    if bad:
        obs[npix // 2, 1, 3] = np.nan
        sig[npix // 3, 2] = 0.0
    return (lines, grids, torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), olines,
            truth)


def _oracle_leg(req, cfg, out):
    """Every served pixel against the oracle: the best parameters decode from
    16-bit genes inside the box, the reported chi-square is the oracle's
    chi-square of those genes within the forward-model bound, and the status
    codes are the oracle's (0 ok, 1 non-finite observation, 2 sigma <= 0)."""
    lines, grids, obs, sig, olines, truth = req
    lo, hi = np.asarray(si.PRIOR_LO), np.asarray(si.PRIOR_HI)
    o64 = obs.cpu().numpy().astype(np.float64)
    s64 = sig.cpu().numpy().astype(np.float64)
    par = out["params"].cpu().numpy()
    chi = out["chi2"].cpu().numpy().astype(np.float64)
    st = out["status"].cpu().numpy()
    ref = oracle.ga_invert(o64, s64, olines, lo, hi, pop=2, generations=0, k=1, p_cross=0.0,
                           p_mut=0.0, seed=0)["status"]
    assert np.array_equal(st, ref)
    ok = st == 0
    assert np.isnan(par[~ok]).all() and np.isnan(chi[~ok]).all()
    genes = recover_genes(par[ok], lo, hi)
    dec = oracle.decode(genes, lo, hi)
    assert np.array_equal(dec.astype(np.float32), par[ok])
    L = o64.shape[-1]
    ref_chi = oracle.chi2(dec[:, None, :], o64[ok], s64[ok], olines)[:, 0]
    models = oracle.me_synth(dec, olines)[:, None]
    tol = chi2_tol(o64[ok], models, s64[ok], ic_of(truth[ok]), 4 * L - 9, FWD_TOL_F32)[:, 0]
    tol += 1e-5 * ref_chi
    assert np.all(np.abs(chi[ok] - ref_chi) <= tol), np.max(np.abs(chi[ok] - ref_chi) / tol)


def _alone(req, cfg):
    lines, grids, obs, sig = req[:4]
    return g.ga_invert(obs, sig, lines, grids, g.bounds(si.PRIOR_LO, si.PRIOR_HI), cfg)


def _same(a, b):
    return (torch.equal(a["params"].nan_to_num(-1), b["params"].nan_to_num(-1))
            and torch.equal(a["chi2"].nan_to_num(-1), b["chi2"].nan_to_num(-1))
            and torch.equal(a["status"], b["status"]))


def _drain(sess, ids, max_steps=500):
    for _ in range(max_steps):
        if all(sess.poll(i) == 1 for i in ids):
            return
        sess.step()
        torch.cuda.synchronize()
    raise AssertionError("requests did not finish")


def test_single_request_equals_ga_invert():
    req = _request("slit", 100, 1, bad=True)
    cfg = g.GAConfig(pop=128, generations=23, seed=5)
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=7)
    rid = sess.submit(req[2], req[3], req[0], req[1], g.bounds(si.PRIOR_LO, si.PRIOR_HI), cfg)
    _drain(sess, [rid])
    out = sess.result(rid)
    assert _same(out, _alone(req, cfg))
    _oracle_leg(req, cfg, out)
    assert sess.stats() == dict(queued=0, resident=0, bytes_in_use=0)
    assert sess.tracked() == 0 and sess.held() == 0
    sess.close()


def test_mixed_requests_equal_their_standalone_runs():
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    reqs = [(_request("tiny", 37, 2), g.GAConfig(pop=64, generations=15, seed=1)),
            (_request("slit", 70, 3, bad=True), g.GAConfig(pop=128, generations=30, seed=2)),
            (_request("slit1", 130, 4), g.GAConfig(pop=96, generations=9, seed=3, pixel_base=7)),
            (_request("tiny", 5, 5), g.GAConfig(pop=2, generations=12, tournament_k=2, seed=4)),
            (_request("slit", 64, 6), g.GAConfig(pop=128, generations=0, seed=6))]
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=4)
    ids = []
    # staggered arrivals: two now, the rest after some steps
    for r, c in reqs[:2]:
        ids.append(sess.submit(r[2], r[3], r[0], r[1], b, c))
    sess.step()
    sess.step()
    for r, c in reqs[2:]:
        ids.append(sess.submit(r[2], r[3], r[0], r[1], b, c))
        sess.step()
    _drain(sess, ids)
    for (r, c), rid in zip(reqs, ids):
        out = sess.result(rid)
        assert _same(out, _alone(r, c)), rid
        _oracle_leg(r, c, out)
    assert sess.tracked() == 0
    sess.close()


def test_budget_admission_and_cancel():
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=128, generations=20, seed=9)
    r1, r2, r3 = _request("tiny", 200, 11), _request("tiny", 150, 12), _request("tiny", 100, 13)
    per_pixel = 128 * (9 * 2 + 4)
    budget = 260 * per_pixel                  # room for one of the larger requests at a time
    sess = g.ServingSession(budget_bytes=budget, gens_per_step=5)
    i1 = sess.submit(r1[2], r1[3], r1[0], r1[1], b, cfg)
    i2 = sess.submit(r2[2], r2[3], r2[0], r2[1], b, cfg)
    i3 = sess.submit(r3[2], r3[3], r3[0], r3[1], b, cfg)
    sess.step()
    st = sess.stats()
    assert st["resident"] == 1 and st["queued"] == 2 and st["bytes_in_use"] <= budget
    sess.cancel(i3)                           # queued: dropped at once
    assert sess.stats()["queued"] == 1 and sess.poll(i3) == -1
    sess.release(i3)
    with pytest.raises(g.GenesisError):       # released: unknown
        sess.poll(i3)
    with pytest.raises(g.GenesisError):       # queued or resident: cannot be released
        sess.release(i2)
    peak = 0
    for _ in range(100):
        sess.step()
        torch.cuda.synchronize()
        peak = max(peak, sess.stats()["bytes_in_use"])
        if sess.poll(i1) == 1 and sess.poll(i2) == 1:
            break
    assert peak <= budget
    assert _same(sess.result(i1), _alone(r1, cfg)) and _same(sess.result(i2), _alone(r2, cfg))
    # a resident request can be cancelled too
    i4 = sess.submit(r1[2], r1[3], r1[0], r1[1], b, cfg)
    sess.step()
    sess.cancel(i4)
    sess.step()
    assert sess.poll(i4) == -1 and sess.stats()["bytes_in_use"] == 0
    sess.release(i4)
    assert sess.tracked() == 0 and sess.held() == 0
    # larger than the whole budget
    big = _request("tiny", 400, 14)
    with pytest.raises(g.GenesisError):
        sess.submit(big[2], big[3], big[0], big[1], b, cfg)
    sess.close()


def test_pixel_cap_admission():
    # a 250-pixel cap: requests of 200, 150 and 100 pixels are admitted one
    # or two at a time in arrival order (a request is always admitted into an
    # empty session, even above the cap), with unchanged results
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=10, seed=21)
    rs = [_request("tiny", 200, 31), _request("tiny", 150, 32), _request("tiny", 100, 33),
          _request("tiny", 300, 34)]
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=5, max_resident_pixels=250)
    ids = [sess.submit(r[2], r[3], r[0], r[1], b, cfg) for r in rs]
    sess.step()
    st = sess.stats()
    assert st["resident"] == 1 and st["queued"] == 3        # 200 + 150 > 250
    resident_seen = []
    for _ in range(100):
        sess.step()
        torch.cuda.synchronize()
        resident_seen.append(sess.stats()["resident"])
        if all(sess.poll(i) == 1 for i in ids):
            break
    assert max(resident_seen) <= 2                          # 150 + 100 fit together
    for r, rid in zip(rs, ids):
        assert _same(sess.result(rid), _alone(r, cfg)), rid
    assert g.lib().gs_set_max_resident_pixels(sess._h, -1) != 0
    assert g.lib().gs_set_max_resident_pixels(None, 10) != 0
    sess.close()


def test_released_requests_leave_no_memory_behind():
    # a long stream of small requests, each fetched when done: the session
    # holds no records or tensors of fetched requests, and the device memory
    # torch has allocated stays flat
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=32, generations=3, seed=3)
    req = _request("tiny", 16, 41)
    sess = g.ServingSession(budget_bytes=1 << 26, gens_per_step=2)
    torch.cuda.synchronize()
    base = None
    for k in range(60):
        # fresh input tensors per request, as a service receiving data would have
        rid = sess.submit(req[2].clone(), req[3].clone(), req[0], req[1], b, cfg)
        _drain(sess, [rid])
        out = sess.result(rid)
        del out
        torch.cuda.synchronize()
        if k == 5:
            base = torch.cuda.memory_allocated()
        if k > 5:
            assert torch.cuda.memory_allocated() <= base, k
    assert sess.tracked() == 0 and sess.held() == 0
    sess.close()


def test_steps_on_alternating_streams():
    # steps issued on two streams alternately: each waits for the previous
    # one, so results equal the standalone inversion
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=64, generations=17, seed=8)
    reqs = [_request("tiny", 40, 51), _request("tiny", 23, 52)]
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=3)
    ids = [sess.submit(r[2], r[3], r[0], r[1], b, cfg) for r in reqs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for k in range(40):
        with torch.cuda.stream(streams[k % 2]):
            sess.step()
    torch.cuda.synchronize()
    assert all(sess.poll(i) == 1 for i in ids)
    for r, rid in zip(reqs, ids):
        assert _same(sess.result(rid), _alone(r, cfg))
    sess.close()


def _fill_request(npix, seed, lo=0.1, hi=1.0):
    lines, grids, olines = [], [], []
    for ln, n in si.line_set("slit"):
        st, sp = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(st, sp, n))
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       st, sp, n))
    c = si.fill_coefficients("slit")
    gf, of = g.fill(lo, hi, *c), oracle.make_fill(lo, hi, *c)
    truth = si.draw_truth(npix, seed)
    alpha = si.draw_alpha(npix, seed)
    obs = oracle.me_synth_fill(truth, alpha, olines, of)
    sig = si.sigma_for(truth)
    obs = (obs + sig[:, :, None] * si.std_normal(obs.shape, seed)).astype(np.float32)
    sig = sig.astype(np.float32)
    obs[npix // 2, 0, 5] = np.nan
    return (lines, grids, torch.tensor(obs, device=DEV), torch.tensor(sig, device=DEV), olines,
            truth, gf, of)


def test_fp16_and_fill_requests_equal_their_standalone_runs():
    # the service runs ga_invert's own generation loop, so FP16-synthesis and
    # fill-fraction requests, mixed with plain ones and arriving late, come
    # out bit-identical to their standalone inversions
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    r16 = _request("slit", 60, 11, bad=True)
    c16 = g.GAConfig(pop=128, generations=17, seed=9, synth_precision=g.SYNTH_FP16)
    rf = _fill_request(50, 12)
    cf = g.GAConfig(pop=96, generations=13, seed=10, init_mode=1, restart_every=5)
    rp = _request("tiny", 20, 13)
    cp = g.GAConfig(pop=64, generations=11, seed=11)
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=5)
    ids = [sess.submit(rp[2], rp[3], rp[0], rp[1], b, cp)]
    sess.step()
    ids.append(sess.submit(r16[2], r16[3], r16[0], r16[1], b, c16))
    ids.append(sess.submit(rf[2], rf[3], rf[0], rf[1], b, cf, fill=rf[6]))
    _drain(sess, ids)
    out_p, out_16, out_f = (sess.result(i) for i in ids)
    assert _same(out_p, _alone(rp, cp))
    assert _same(out_16, _alone(r16, c16))
    alone_f = g.ga_invert(rf[2], rf[3], rf[0], rf[1], b, cf, fill=rf[6])
    assert _same(out_f, alone_f)
    assert torch.equal(out_f["alpha"].nan_to_num(-1), alone_f["alpha"].nan_to_num(-1))
    # oracle leg of the fill request: status, and the reported chi-square and
    # alpha are the oracle's fill merit and best alpha of the decoded genes
    lines, grids, obs, sig, olines, truth, gf, of = rf
    lo, hi = np.asarray(si.PRIOR_LO), np.asarray(si.PRIOR_HI)
    st = out_f["status"].cpu().numpy()
    ok = st == 0
    assert st[~ok].tolist() == [1] and np.isnan(out_f["alpha"].cpu().numpy()[~ok]).all()
    par = out_f["params"].cpu().numpy()[ok]
    dec = oracle.decode(recover_genes(par, lo, hi), lo, hi)
    o64 = obs.cpu().numpy().astype(np.float64)[ok]
    s64 = sig.cpu().numpy().astype(np.float64)[ok]
    ref, aref = oracle.chi2_fill(dec[:, None, :], o64, s64, olines, of)
    chi = out_f["chi2"].cpu().numpy().astype(np.float64)[ok]
    L = o64.shape[-1]
    models = np.stack([oracle.me_synth_fill(dec[i:i + 1], aref[i], olines, of)[0]
                       for i in range(len(dec))])
    delta = FWD_TOL_F32 * ic_of(dec)[:, None, None]
    rr = np.abs(o64 - models)
    w2 = 1.0 / s64[:, :, None] ** 2
    bound = (w2 * (2 * rr * delta + delta ** 2)).sum(axis=(1, 2)) / (4 * L - 10)
    assert np.all(np.abs(chi - ref[:, 0]) <= bound + 1e-5 * ref[:, 0])
    da = np.abs(out_f["alpha"].cpu().numpy()[ok] - aref[:, 0])
    assert np.median(da) <= 1e-5 and da.max() <= 1e-3, da
    # the FP16 request's oracle leg: status and decodable parameters (its
    # fitness is the FP16 synthesis's, checked against the oracle in the FP16
    # tests)
    st16 = out_16["status"].cpu().numpy()
    ref16 = oracle.ga_invert(r16[2].cpu().numpy().astype(np.float64),
                             r16[3].cpu().numpy().astype(np.float64), r16[4], lo, hi, pop=2,
                             generations=0, k=1, p_cross=0.0, p_mut=0.0, seed=0)["status"]
    assert np.array_equal(st16, ref16)
    sess.close()


def test_fp16_fill_request_equals_its_standalone_run():
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    rf = _fill_request(40, 14)
    cfg = g.GAConfig(pop=64, generations=12, seed=13, synth_precision=g.SYNTH_FP16)
    sess = g.ServingSession(budget_bytes=1 << 30, gens_per_step=5)
    rid = sess.submit(rf[2], rf[3], rf[0], rf[1], b, cfg, fill=rf[6])
    _drain(sess, [rid])
    out = sess.result(rid)
    alone = g.ga_invert(rf[2], rf[3], rf[0], rf[1], b, cfg, fill=rf[6])
    assert _same(out, alone)
    assert torch.equal(out["alpha"].nan_to_num(-1), alone["alpha"].nan_to_num(-1))
    sess.close()
