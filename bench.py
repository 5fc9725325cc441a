"""Benchmark: GA Milne-Eddington inversion of a synthetic full-disc map on one MI355X.

Default workload ('disc'): the on-disc pixels of a 2048 x 2048 map (3,294,288
pixels; smooth random parameter fields plus strong-field patches, mu from the
disc position) x 2 lines (Fe I 6301.5 full 12-component pattern, Fe I 6302.5
triplet) x 128 samples over +-0.4 A; FP32 GA with population 128, 150
generations, tournament 4, mutation rate 0.05, crossover 0.85, then 10 FP64
Levenberg-Marquardt iterations polishing each pixel's best individual.  The
map is split into 20 contiguous scanline blocks of equal pixel count; one step
inverts one block (one ga_invert launch with pixel_base = the block's first
pixel, so every pixel draws the random numbers it would in a single launch,
then one me_refine_f64 launch), so 20 steps invert the whole disc once.
Observations are noise-free (the accuracy gate, p90 |dB| <= 10 G, is defined
on noise-free truth), synthesised on the device by the FP64 forward model
before the timed region (the CPU-baseline leg compares those of its sample
pixels with the oracle's; tests/test_gpu_disc.py checks a block against the
oracle); the GA reads them rounded to FP32.  Inputs are resident in HBM
before the timed region.  Prints ONE JSON line.

Other workloads: 'slit' (2048 px, G 200), 'tiny' (64 px, FP64), 'precision'
(FP32 against FP16 synthesis on a strided disc sample, noisy), 'serving',
'proposal', 'fill'.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel inversions/s at fixed param accuracy; ME evals/s vs VALU peak; p99 tile ms"

# Algorithmic FP32 work of the implemented formulas (FMA = 2 flops, reciprocal
# = 1): per Zeeman component and wavelength (reduced wavelength, rational
# Faddeeva in v^2, accumulation) and per wavelength (propagation matrix,
# Unno-Rachkovsky closed form, chi-square terms).
FLOP_PER_COMP_LAMBDA = 42
FLOP_PER_LAMBDA = 71
PEAK_FP32_VALU = 157.3e12     # MI355X published FP32 vector peak (reached without packed
                              # instructions: two-operand VOP2 FP32 issues in about 2 cycles)
PEAK_FP64_VALU = 78.6e12


# FP64 Levenberg-Marquardt iterations after the GA: the fewest that keep the
# slit row inside the accuracy gate (p90 |dB| <= 10 G on noise-free truth)
# with margin -- p90 |dB| 8.4 G after 5, 3.6 G after 10, 0.66 G after 50.
REFINE_ITERS = 10

# HBM bytes per launch of k_ga_invert<float> from the FETCH_SIZE and
# WRITE_SIZE counters scaled by a device copy of known size (profiles/
# k_ga_invert_disc_counters.md): one full-disc block, and the slit row.  Valid
# only for the machine code they were measured on: reported while the build's
# code hash of that kernel (libgenesis_hip.layout.json) equals this one.
TRAFFIC_DISC_BLOCK_BYTES = 18.607e9
TRAFFIC_SLIT_BYTES = 243.08e6
TRAFFIC_CODE_SHA256 = "568e627056b42b8948b3f83600d315b51575a9ab2660813ccb14e1154b399a9b"


def measured_traffic(nbytes):
    """nbytes while the installed k_ga_invert<float> is the measured one, else None."""
    from paper_1208_0302_amd import build as gbuild
    rec = gbuild.layout().get("GENESIS_PAD_INVERT_F32", {})
    if nbytes is None or TRAFFIC_CODE_SHA256 is None or \
            rec.get("code_sha256") != TRAFFIC_CODE_SHA256:
        return None
    return nbytes


def disc_traffic(edges):
    return measured_traffic(TRAFFIC_DISC_BLOCK_BYTES)


def workload(name):
    if name == "slit":
        return dict(name=name, npix=2048, lines="slit", pop=128, generations=200, k=4,
                    p_mut=0.05, p_cross=0.85, seed=0, dtype="f32", refine=REFINE_ITERS)
    if name == "tiny":
        return dict(name=name, npix=64, lines="tiny", pop=64, generations=100, k=4,
                    p_mut=0.05, p_cross=0.85, seed=0, dtype="f64", refine=REFINE_ITERS)
    raise SystemExit("unknown workload %s" % name)


def flops_per_eval(lines):
    f = 0
    for ln, g in lines:
        f += g.n * (ln.ncomp * FLOP_PER_COMP_LAMBDA + FLOP_PER_LAMBDA)
    return f


def describe(w, lines):
    parts = []
    for ln, g in lines:
        parts.append("%.4f A (%d comp) x %d" % (ln.lambda0_A, ln.ncomp, g.n))
    return ("%s: %d px x [%s], pop %d, G %d, k %d, p_mut %.2f, p_cross %.2f, %s GA + "
            "%d FP64 Levenberg-Marquardt iterations"
            % (w["name"], w["npix"], "; ".join(parts), w["pop"], w["generations"], w["k"],
               w["p_mut"], w["p_cross"], w["dtype"].upper(), w["refine"]))


def cpu_baseline(w, truth, line_set, budget_s=20.0, mu=None, device_obs=None):
    """The FP64 oracle's GA on a bounded sample of the same workload, on the
    host cores: `nthr` pixels of `truth` (their observations synthesised by
    the oracle itself, with mu if given), generations chosen so the run takes
    roughly `budget_s`; scaled to full inversions per second.  device_obs
    (the benchmark's observations of the same pixels, FP64 [n, 4, L]) are
    compared with the oracle's, relative to the continuum."""
    import oracle
    import synth_inputs as si
    olines = []
    for ln, n in si.line_set(line_set):
        start, step = si.grid(ln, n)
        olines.append(oracle.make_line(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"],
                                       start, step, n))
    nthr = oracle.num_threads()
    npx = min(max(nthr, 1), len(truth))
    m = None if mu is None else mu[:npx]
    obs_np = oracle.me_synth(truth[:npx], olines, m)
    sig_np = si.sigma_for(truth[:npx], mu=m)
    cert = None
    if device_obs is not None:
        ic = (truth[:npx, 7] + (1.0 if m is None else m) * truth[:npx, 8])[:, None, None]
        cert = float(np.max(np.abs(np.asarray(device_obs)[:npx] - obs_np) / ic))
    # probe: one generation
    t0 = time.perf_counter()
    oracle.ga_invert(obs_np[:npx], sig_np[:npx], olines, si.PRIOR_LO, si.PRIOR_HI,
                     pop=w["pop"], generations=0, k=w["k"], p_cross=w["p_cross"],
                     p_mut=w["p_mut"], seed=w["seed"], mu=m)
    t_gen = time.perf_counter() - t0
    gs = int(max(0, min(w["generations"], budget_s / max(t_gen, 1e-6) - 1)))
    t0 = time.perf_counter()
    ga = oracle.ga_invert(obs_np[:npx], sig_np[:npx], olines, si.PRIOR_LO, si.PRIOR_HI,
                          pop=w["pop"], generations=gs, k=w["k"], p_cross=w["p_cross"],
                          p_mut=w["p_mut"], seed=w["seed"], mu=m)
    dt_ga = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.lm_refine(obs_np[:npx], sig_np[:npx], olines, si.PRIOR_LO, si.PRIOR_HI,
                     ga["params"], w["refine"], mu=m)
    dt_lm = time.perf_counter() - t0
    t_full = dt_ga * (w["generations"] + 1) / (gs + 1) + dt_lm
    out = {"value": npx / t_full, "unit": "pixels/s", "cores": nthr, "kind": "oracle",
           "sample": "%d pixels of the %s workload: %d of %d GA generations (pop %d, %.1f s, "
                     "scaled by (G+1)) plus %d LM iterations (%.1f s), FP64 oracle with "
                     "OpenMP over pixels"
                     % (npx, w["name"], gs + 1, w["generations"] + 1, w["pop"], dt_ga,
                        w["refine"], dt_lm)}
    if cert is not None:
        out["observations_vs_oracle_max_over_Ic"] = cert
    return out


def serving(args):
    """Continuous-batching service under a Poisson stream of inversion
    requests (tiles of lognormal size, 1-2 lines x 128 samples, 50-300
    generations, population 128, 200 GB budget).  Latency = arrival to
    outputs complete on the device, at launch granularity."""
    import torch
    import paper_1208_0302_amd as g
    import synth_inputs as si

    dev = torch.device("cuda:0")
    sched = si.serving_schedule(args.rate, args.window, seed=0, median_px=args.tile_median,
                                min_px=min(256, int(args.tile_median)))
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    linesets = {}
    for name in ("slit", "slit1"):
        ls, gs = [], []
        for ln, n in si.line_set(name):
            start, step = si.grid(ln, n)
            ls.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
            gs.append(g.grid(start, step, n))
        linesets[name] = (ls, gs)
    # observations of every request synthesised up front (resident before arrival)
    reqs = []
    for k, r in enumerate(sched):
        ls, gs = linesets[r["lines"]]
        truth = si.draw_truth(r["npix"], seed=r["seed"])
        obs = g.me_synth(torch.tensor(truth, dtype=torch.float32, device=dev), ls, gs)
        sig = torch.tensor(si.sigma_for(truth), dtype=torch.float32, device=dev)
        reqs.append(dict(r, obs=obs, sig=sig, ls=ls, gs=gs))
    torch.cuda.synchronize()
    print("serving: %d requests, %d pixels synthesised" % (len(reqs), sum(r["npix"] for r in reqs)),
          file=sys.stderr, flush=True)
    sess = g.ServingSession(budget_bytes=200 * 10 ** 9, gens_per_step=args.gens_per_step,
                            max_resident_pixels=args.max_resident_pixels)
    pending, lat, done_px, launches = {}, [], 0, 0
    nxt = 0
    t0 = time.perf_counter()
    last = t0
    while nxt < len(reqs) or pending:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt]["t"] <= now:
            r = reqs[nxt]
            cfg = g.GAConfig(pop=128, generations=r["generations"], tournament_k=4,
                             p_cross=0.85, p_mut=0.05, seed=r["seed"])
            rid = sess.submit(r["obs"], r["sig"], r["ls"], r["gs"], b, cfg)
            pending[rid] = r
            nxt += 1
        if not pending:
            time.sleep(min(0.002, max(0.0, reqs[nxt]["t"] - now)))
            continue
        sess.step()
        torch.cuda.synchronize()
        launches += 1
        tnow = time.perf_counter() - t0
        for rid in [i for i in pending if sess.poll(i) == 1]:
            sess.release(rid)
            r = pending.pop(rid)
            lat.append(tnow - r["t"])
            done_px += r["npix"]
        if time.perf_counter() - last > 5.0:
            last = time.perf_counter()
            print("serving: t=%.1f s, done %d, pending %d, queued %d" %
                  (tnow, len(lat), len(pending), sess.stats()["queued"]), file=sys.stderr,
                  flush=True)
    makespan = time.perf_counter() - t0
    sess.close()
    lat = np.array(lat)
    # the plain GA on the same stream: a first-come-first-served loop that runs
    # each request's ga_invert to completion before taking the next (the same
    # results: each service result equals its standalone inversion)
    lat_p, done_p = [], 0
    t0 = time.perf_counter()
    last = t0
    for r in reqs:
        now = time.perf_counter() - t0
        if r["t"] > now:
            time.sleep(r["t"] - now)
        cfg = g.GAConfig(pop=128, generations=r["generations"], tournament_k=4,
                         p_cross=0.85, p_mut=0.05, seed=r["seed"])
        g.ga_invert(r["obs"], r["sig"], r["ls"], r["gs"], b, cfg, want_status=False)
        torch.cuda.synchronize()
        lat_p.append(time.perf_counter() - t0 - r["t"])
        done_p += r["npix"]
        if time.perf_counter() - last > 5.0:
            last = time.perf_counter()
            print("serving (plain loop): t=%.1f s, done %d" % (last - t0, len(lat_p)),
                  file=sys.stderr, flush=True)
    makespan_p = time.perf_counter() - t0
    lat_p = np.array(lat_p)
    out = {"metric": METRIC + " (serving)", "value": done_px / makespan, "unit": "pixels/s",
           "n_gpus": 1, "steps": launches, "warmup": 0, "ms_per_step": makespan * 1e3 / launches,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (Poisson request stream, truth from the priors)",
           "config": {"workload": "serving: Poisson %.2f req/s over %.0f s, tiles "
                                  "clip(lognormal(ln %g, 1.2), %d, 65536) px, 1-2 lines x 128, "
                                  "G ~ U{50..300}, pop 128, %d generations per launch, 200 GB "
                                  "budget, resident-pixel cap %s"
                                  % (args.rate, args.window, args.tile_median,
                                     min(256, int(args.tile_median)), args.gens_per_step,
                                     args.max_resident_pixels or "none"),
                      "requests": len(reqs)},
           "latency_s_p50": float(np.percentile(lat, 50)),
           "latency_s_p99": float(np.percentile(lat, 99)),
           "makespan_s": makespan,
           "plain_fcfs": {"pixels_per_s": done_p / makespan_p,
                          "latency_s_p50": float(np.percentile(lat_p, 50)),
                          "latency_s_p99": float(np.percentile(lat_p, 99)),
                          "makespan_s": makespan_p},
           "speedup_vs_plain": (done_px / makespan) / (done_p / makespan_p)}
    print(json.dumps(out), flush=True)


# Algorithmic matrix-product work of one training example of the proposal
# network (1024 -> 512 -> 512 -> 512 -> 9): forward, weight gradients, and the
# input gradients of the three upper layers (FMA = 2 flops).
MLP_DIMS = (1024, 512, 512, 512, 9)
MLP_FWD_FLOP = 2 * sum(MLP_DIMS[i] * MLP_DIMS[i + 1] for i in range(4))
MLP_TRAIN_FLOP = 2 * MLP_FWD_FLOP + 2 * sum(MLP_DIMS[i] * MLP_DIMS[i + 1] for i in range(1, 4))
PEAK_BF16_MFMA = 2.5e15       # MI355X published dense BF16 matrix peak


def proposal(args):
    """Learned proposal: BF16 training of the network on examples synthesised
    on the fly (one step = one mlp_train step of `batch` examples: draw,
    me_synth, noise, features, forward, backward, Adam), then the comparison
    of initial populations on held-out noisy pixels: median chi-square and the
    fraction of pixels at or below the reduced chi-square target after G
    generations (and after G = 200 plus the FP64 refinement), for a random
    population, 32 of 128 individuals seeded from the network (1 exact + 31
    jittered), 32 seeded from the physics first guesses (me_first_guess: B,
    inclination and v_los), Sobol points, Sobol points with restarts every
    50 generations (G/4 of the 200-generation run, Sec. 5.6), and random
    populations searched in per-pixel boxes (me_search_box): the V-lobe
    polarity alone, with the ranges of the non-magnetic pre-fit
    (me_prefit_f64), and those boxes with the physics seeds inside them."""
    import torch
    import paper_1208_0302_amd as g
    import synth_inputs as si

    dev = torch.device("cuda:0")
    batch, lr = args.batch, args.lr
    lines, grids = [], []
    for ln, n in si.line_set("slit"):
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    net = g.MLP(seed=0, device=dev)
    for i in range(args.warmup):
        net.train(lines, grids, b, steps=1, batch=batch, lr=lr, seed=1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    chunk = max(1, args.steps // 10)
    done, losses = 0, []
    while done < args.steps:
        n = min(chunk, args.steps - done)
        losses.append(net.train(lines, grids, b, steps=n, batch=batch, lr=lr, seed=1))
        done += n
        torch.cuda.synchronize()
        print("proposal: %d/%d training steps, loss %.4f" % (done, args.steps,
                                                             losses[-1][-1].item()),
              file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    train_ms = e0.elapsed_time(e1)
    losses = torch.cat(losses).cpu().numpy()

    # one gradient pass (all matrix products of a step) timed on its own
    x, t = net.examples(99, 0, batch, lines, grids, b)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 20
    ev[0].record(stream)
    for _ in range(reps):
        net.compute_grad(x, t)
    ev[1].record(stream)
    torch.cuda.synchronize()
    pass_s = ev[0].elapsed_time(ev[1]) / reps / 1e3
    pass_flop = batch * MLP_TRAIN_FLOP
    res = _heldout(args, g, si, net, lines, grids, b, stream, dev)
    _proposal_report(args, g, si, batch, lr, wall, train_ms, losses, pass_flop, pass_s, *res)


# one strategy per Sec. 5.5 seed (me_seeds order), each alone in 32 slots
SEED_STRATEGIES = ("seed_weak_field", "seed_integral", "seed_cog", "seed_nonmagnetic")


def _heldout(args, g, si, net, lines, grids, b, stream, dev):
    """Initial-population strategies on held-out noisy pixels: median
    chi-square and fraction at the target after G generations."""
    import torch
    npix = args.heldout
    truth = si.draw_truth(npix, seed=123)
    obs = g.me_synth(torch.tensor(truth, dtype=torch.float32, device=dev), lines, grids)
    sig_np = si.sigma_for(truth)
    sig = torch.tensor(sig_np, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(123)
    obs += sig[:, :, None] * torch.randn(obs.shape, generator=gen, device=dev)
    ei = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ei[0].record(stream)
    guess = net.predict(obs, grids, b)
    ei[1].record(stream)
    torch.cuda.synchronize()
    infer_ms = ei[0].elapsed_time(ei[1])
    target = args.chi2_target
    wanted = args.strategies.split(",")
    need_phys = any(w in ("physics", "polarity_box", "prefit_box", "physics_in_box")
                    or w in SEED_STRATEGIES or w.startswith("four_seeds") for w in wanted)
    obs64 = obs.double().contiguous() if need_phys else None
    sig64 = sig.double().contiguous() if need_phys else None
    phys = box_pf = box_pol = None
    box_stats = None
    seeds = seeds_pol = None
    if need_phys:
        phys, box_pf, box_pol, box_stats = _physics_inputs(g, si, obs64, sig64, lines, grids, b,
                                                           truth, stream)
        es = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        es[0].record(stream)
        seeds = g.me_seeds(obs64, lines, grids, b)
        es[1].record(stream)
        seeds_pol = g.me_seeds(obs64, lines, grids, b, pixel_bounds=box_pol)
        torch.cuda.synchronize()
        box_stats["seeds_ms"] = es[0].elapsed_time(es[1])
        sp = seeds.cpu().numpy()
        box_stats["seed_errors"] = {
            name: {"p50_abs_dB_G": float(np.median(np.abs(sp[:, k, 0] - truth[:, 0]))),
                   "p50_abs_dincl_deg_B_ge_300G": (float(np.median(np.abs(
                       sp[truth[:, 0] >= 300, k, 1] - truth[truth[:, 0] >= 300, 1])))
                       if k < 3 else None)}
            for k, name in enumerate(g.SEED_NAMES)}
        print("proposal: Sec. 5.5 seeds %s" % box_stats["seed_errors"], file=sys.stderr,
              flush=True)
    one = {name: dict(n_seeded=32, seed_jitter=512,
                      seed_params=None if seeds is None else seeds[:, k].contiguous())
           for k, name in enumerate(SEED_STRATEGIES)}
    strategies = tuple((n, e) for n, e in (
        ("random", {}),
        ("seeded", dict(n_seeded=32, seed_jitter=512, seed_params=guess)),
        ("physics", dict(n_seeded=32, seed_jitter=512, seed_params=phys)),
        ("polarity_box", dict(pixel_bounds=box_pol)),
        ("prefit_box", dict(pixel_bounds=box_pf)),
        ("physics_in_box", dict(n_seeded=32, seed_jitter=512, seed_params=phys,
                                pixel_bounds=box_pf)),
        ("sobol", dict(init_mode=1)),
        ("sobol_restart", dict(init_mode=1, restart_every=50)),
        *((n, one[n]) for n in SEED_STRATEGIES),
        ("four_seeds", dict(n_seeded=32, seed_jitter=512, seed_params=seeds)),
        ("four_seeds_polarity", dict(n_seeded=32, seed_jitter=512, seed_params=seeds_pol,
                                     pixel_bounds=box_pol)),
        # as Sec. 5.5 places them: each first guess once, exactly, among an
        # otherwise random population
        ("four_seeds_exact", dict(n_seeded=4, seed_jitter=0, seed_params=seeds)),
        ("four_seeds_exact_polarity", dict(n_seeded=4, seed_jitter=0, seed_params=seeds_pol,
                                           pixel_bounds=box_pol))) if n in wanted)
    table = []
    o64, s64 = obs.double(), sig.double()
    for gens in (0, 10, 25, 50, 100, 150, 200):
        row = {"generations": gens}
        for name, extra in strategies:
            cfg = g.GAConfig(pop=128, generations=gens, tournament_k=4, p_cross=0.85,
                             p_mut=0.05, seed=7, **extra)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record(stream)
            r = g.ga_invert(obs, sig, lines, grids, b, cfg)
            ev[1].record(stream)
            ref = g.me_refine_f64(o64, s64, lines, grids, b, r["params"].double().contiguous(),
                                  REFINE_ITERS)
            ev[2].record(stream)
            c = r["chi2"].cpu().numpy()
            cr = ref["chi2"].cpu().numpy()
            row[name + "_median_chi2"] = float(np.median(c))
            row[name + "_frac_at_target"] = float((c <= target).mean())
            row[name + "_refined_median_chi2"] = float(np.median(cr))
            row[name + "_refined_frac_at_target"] = float((cr <= target).mean())
            row[name + "_ga_ms"] = ev[0].elapsed_time(ev[1])
            row[name + "_refine_ms"] = ev[1].elapsed_time(ev[2])
            del ref, r
        table.append(row)
        print("proposal: G=%d %s" % (gens, row), file=sys.stderr, flush=True)
    return table, strategies, box_stats, infer_ms, guess, truth, npix


def _physics_inputs(g, si, obs64, sig64, lines, grids, b, truth, stream):
    """Physics first guesses (weak-field, centre-of-gravity) for B,
    inclination and v_los (NaN elsewhere), and the per-pixel search boxes:
    the V-lobe polarity alone, and with the ranges of the non-magnetic
    pre-fit (Sec. 5.3, 5.5)."""
    import torch
    ef = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ef[0].record(stream)
    guess9 = g.me_first_guess(obs64, lines, grids, b)
    ef[1].record(stream)
    phys = guess9.clone()
    phys[:, [2, 4, 5, 6, 7, 8]] = float("nan")
    eb = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    eb[0].record(stream)
    pre = g.me_prefit_f64(obs64, sig64, lines, grids, b, guess9.double().contiguous(), 20)
    eb[1].record(stream)
    box_pf = g.me_search_box(obs64, sig64, lines, grids, b, prefit=pre["params"],
                             polarity_nsigma=3.0)
    eb[2].record(stream)
    box_pol = g.me_search_box(obs64, sig64, lines, grids, b, polarity_nsigma=3.0)
    torch.cuda.synchronize()
    prefit_ms, box_ms = eb[0].elapsed_time(eb[1]), eb[1].elapsed_time(eb[2])
    bp = box_pf.cpu().numpy()
    inside = (truth >= bp[:, 0]) & (truth <= bp[:, 1])
    box_stats = {"first_guess_ms": ef[0].elapsed_time(ef[1]), "prefit_ms": prefit_ms,
                 "search_box_ms": box_ms,
                 "polarity_restricted_frac": float(((bp[:, 1, 1] - bp[:, 0, 1]) <= 90.0).mean()),
                 "truth_inside_frac": {si.PARAM_NAMES[j]: float(inside[:, j].mean())
                                       for j in (1, 4, 5, 6, 8)},
                 "median_width_frac": {si.PARAM_NAMES[j]: float(np.median(
                     (bp[:, 1, j] - bp[:, 0, j]) / (si.PRIOR_HI[j] - si.PRIOR_LO[j])))
                     for j in (1, 4, 5, 6, 8)}}
    print("proposal: search boxes %s" % box_stats, file=sys.stderr, flush=True)
    return phys, box_pf, box_pol, box_stats


def _equal_accuracy(table, strategies, infer_ms, box_stats):
    if not any(n == "random" for n, _ in strategies):
        return None
    # preparation each strategy needs before its search
    fg = box_stats["first_guess_ms"] if box_stats else 0.0
    pf = (box_stats["prefit_ms"] + box_stats["search_box_ms"]) if box_stats else 0.0
    sd = box_stats.get("seeds_ms", 0.0) if box_stats else 0.0
    prep = {"seeded": infer_ms, "physics": fg,
            "polarity_box": box_stats["search_box_ms"] if box_stats else 0.0,
            "prefit_box": fg + pf, "physics_in_box": fg + pf, "four_seeds": sd,
            "four_seeds_polarity": sd + (box_stats["search_box_ms"] if box_stats else 0.0)}
    prep.update({n: sd for n in SEED_STRATEGIES})
    last = table[-1]
    goal = last["random_refined_frac_at_target"]
    t_random = last["random_ga_ms"] + last["random_refine_ms"]
    out = {"random_generations": last["generations"], "random_refined_frac_at_target": goal,
           "random_ms": t_random}
    for n, extra in strategies:
        row = next((r for r in table if r[n + "_refined_frac_at_target"] >= goal), None)
        if row is None:
            out[n] = None
            continue
        t = row[n + "_ga_ms"] + row[n + "_refine_ms"] + prep.get(n, 0.0)
        out[n] = {"generations": row["generations"], "ms": t, "speedup": t_random / t,
                  "refined_frac_at_target": row[n + "_refined_frac_at_target"]}
    return out


def _proposal_report(args, g, si, batch, lr, wall, train_ms, losses, pass_flop, pass_s, table,
                     strategies, box_stats, infer_ms, guess, truth, npix):
    target = args.chi2_target

    def first_reaching(name):
        for row in table:
            if row[name + "_median_chi2"] <= target:
                return row["generations"]
        return None

    gp = guess.cpu().numpy()
    err = np.abs(gp - truth)
    err[:, 2] = np.minimum(err[:, 2], 180.0 - err[:, 2])
    out = {"metric": "proposal training examples/s (BF16 matrix cores, FP32 master weights)",
           "value": batch * args.steps / wall, "unit": "examples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic (examples drawn from the priors and synthesised on the device; "
                   "held-out pixels from an independent generator, noise 1e-3 Ic)",
           "config": {"workload": "learned proposal: MLP 1024-512-512-512-9 GELU, batch %d, "
                                  "Adam lr %g; held-out %d px x 2 lines x 128, pop 128, "
                                  "32 seeded (1 exact + 31 jittered +-512 codes)"
                                  % (batch, lr, npix), "batch": batch, "heldout": npix},
           "train_ms_device": train_ms,
           "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-10:].mean()),
           "inference_ms": infer_ms, "inference_px_per_s": npix / (infer_ms / 1e3),
           "proposal_median_abs_err": dict(zip(si.PARAM_NAMES,
                                               np.median(err, axis=0).round(4).tolist())),
           "chi2_target": target,
           "generations_to_median_target": {n: first_reaching(n) for n, _ in strategies},
           # the first checkpoint at which each strategy's median chi-square is at or
           # below the random population's after the last generation
           # equal accuracy: the fewest generations after which GA + refinement puts
           # at least as many pixels at the target as the random population's last
           # checkpoint does, and the time ratio (the seeded forms include inference)
           "equal_accuracy_vs_random": _equal_accuracy(table, strategies, infer_ms, box_stats),
           "generations_to_random_final_median": {
               n: next((row["generations"] for row in table
                        if row[n + "_median_chi2"] <= table[-1]["random_median_chi2"]), None)
               for n, _ in strategies} if any(n == "random" for n, _ in strategies) else None,
           "search_boxes": box_stats,
           "seeding_table": table,
           "roofline": {"bound": "mfma", "achieved": pass_flop / pass_s / 1e12,
                        "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                        "frac": pass_flop / pass_s / PEAK_BF16_MFMA, "traffic": None,
                        "kernel": "mlp_grad pass (ten launches: k_prep, k_mm forward, "
                                  "output, backward and weight-gradient products, "
                                  "k_grad_reduce)",
                        "flop_per_example": MLP_TRAIN_FLOP, "examples_per_launch": batch}}
    print(json.dumps(out), flush=True)


def precision_study(args):
    """Precision study on the full-disc configuration: on-disc pixels of a
    2048 x 2048 map (every `disc_stride`-th), parameters from smooth random
    fields plus strong-field patches, mu from the disc position, 2 lines x
    128 samples, noise 1e-3 Ic; population 128, 150 generations.  The GA runs
    with FP32 synthesis and with packed-FP16 profile synthesis (FP32
    chi-square); each is followed by REFINE_ITERS FP64 Levenberg-Marquardt
    iterations.
    One step = GA + refinement of every pixel of the sample, FP16 synthesis."""
    import torch
    import paper_1208_0302_amd as g
    import synth_inputs as si

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    truth, mu_np, _ = si.full_disc(2048, seed=0, stride=args.disc_stride)
    npix = truth.shape[0]
    print("disc: %d on-disc pixels sampled (%.1f s)" % (npix, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    lines, grids = [], []
    for ln, n in si.line_set("slit"):
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
    mu = torch.tensor(mu_np, dtype=torch.float32, device=dev)
    obs = g.me_synth(torch.tensor(truth, dtype=torch.float32, device=dev), lines, grids, mu=mu)
    sig_np = si.sigma_for(truth, mu=mu_np)
    sig = torch.tensor(sig_np, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(20480)
    obs += sig[:, :, None] * torch.randn(obs.shape, generator=gen, device=dev)
    obs64, sig64, mu64 = obs.double(), sig.double(), mu.double()
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)

    def errors(params):
        d = np.abs(params - truth)
        d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
        strong = truth[:, 0] >= 500.0
        out = {}
        for j, name in enumerate(si.PARAM_NAMES):
            sel = strong if name in ("incl", "azim") else slice(None)
            out[name] = {"p50": float(np.percentile(d[sel, j], 50)),
                         "p90": float(np.percentile(d[sel, j], 90))}
        return out

    rows, times = {}, {}
    for name, sp in (("fp32", g.SYNTH_NATIVE), ("fp16", g.SYNTH_FP16)):
        cfg = g.GAConfig(pop=128, generations=150, tournament_k=4, p_cross=0.85, p_mut=0.05,
                         seed=0, synth_precision=sp)
        g.ga_invert(obs[:256], sig[:256], lines, grids, b, cfg, mu=mu[:256])   # warm-up
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        w0 = time.perf_counter()
        ev[0].record(stream)
        r = g.ga_invert(obs, sig, lines, grids, b, cfg, mu=mu)
        ev[1].record(stream)
        ref = g.me_refine_f64(obs64, sig64, lines, grids, b, r["params"].double().contiguous(),
                              REFINE_ITERS, mu=mu64)
        ev[2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        times[name] = {"ga_ms": ev[0].elapsed_time(ev[1]), "refine_ms": ev[1].elapsed_time(ev[2]),
                       "wall_s": wall}
        rows[name + "_ga"] = errors(r["params"].double().cpu().numpy())
        rows[name + "_ga_refine"] = errors(ref["params"].cpu().numpy())
        rows[name + "_ga"]["median_chi2"] = float(r["chi2"].median().item())
        rows[name + "_ga_refine"]["median_chi2"] = float(ref["chi2"].median().item())
        print("disc: %s GA %.1f ms, refine %.1f ms" % (name, times[name]["ga_ms"],
                                                      times[name]["refine_ms"]),
              file=sys.stderr, flush=True)
    lines_grids = list(zip(lines, grids))
    evals = npix * 128 * 151
    fpe = flops_per_eval(lines_grids)
    # the counted FP32 work of the degree-7 formula over the FP32 kernel's
    # time (the FP16 kernel evaluates a different, degree-4 rational)
    ga_s = times["fp32"]["ga_ms"] / 1e3
    out = {"metric": "pixel inversions/s, full-disc precision study (FP16 synthesis + FP64 refine)",
           "value": npix / times["fp16"]["wall_s"], "unit": "pixels/s", "n_gpus": 1, "steps": 1,
           "warmup": 1, "ms_per_step": times["fp16"]["wall_s"] * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f16",
           "data": "synthetic (smooth random parameter fields + strong-field patches on a "
                   "2048^2 disc, mu from the disc position, noise 1e-3 Ic)",
           "config": {"workload": "precision study: full disc 2048^2 (every %d-th of the on-disc pixels), "
                                  "2 lines x 128, pop 128, G 150, FP32 vs FP16 synthesis, "
                                  "FP32 chi-square, %d FP64 L-M iterations"
                                  % (args.disc_stride, REFINE_ITERS),
                      "npix": npix},
           "fp32_pixels_per_s": npix / times["fp32"]["wall_s"],
           "times_ms": times,
           "error_table": rows,
           "timed_pixels": npix,
           "roofline": {"bound": "alu", "achieved": evals * fpe / ga_s / 1e12,
                        "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                        "frac": evals * fpe / ga_s / PEAK_FP32_VALU, "traffic": None,
                        "kernel": "k_ga_invert<float> (FP32 synthesis)",
                        "flop_per_eval": fpe, "evals_per_launch": evals}}
    print(json.dumps(out), flush=True)


# FP32 flops per wavelength that the fill fraction adds to an evaluation
# (Sec. 5.2): the field-free profile (offset 4, Voigt H 42, N 2), D_I 2, and
# the three weighted sums e.e, e.D, D.D (36) in place of the plain
# chi-square's 12.
FLOP_FILL_PER_LAMBDA = 4 + 42 + 2 + 2 + 36 - 12


def fill_workload(args):
    """Fill fraction (Sec. 5.2): 2048 slit pixels whose magnetic fraction alpha
    is drawn from U(0.25, 1), mu from U(0.3, 1), mixed with the field-free
    stand-in profile (FILL_CLV), noise 1e-3 Ic.  The GA with the fill fraction
    (alpha in [0, 1] solved per individual) against the plain GA on the same
    observations: time, alpha and field-strength errors."""
    import torch
    import paper_1208_0302_amd as g
    import synth_inputs as si

    dev = torch.device("cuda:0")
    npix = 2048
    lines, grids = [], []
    for ln, n in si.line_set("slit"):
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
    fill = g.fill(0.0, 1.0, *si.fill_coefficients("slit"))
    truth = si.draw_truth(npix, 77)
    alpha = si.draw_alpha(npix, 77)
    mu_np = np.random.default_rng(78).uniform(0.3, 1.0, npix)
    t32 = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)
    mu = t32(mu_np)
    obs = g.me_synth(t32(truth), lines, grids, mu=mu, alpha=t32(alpha), fill=fill)
    sig_np = si.sigma_for(truth, mu=mu_np)
    sig = t32(sig_np)
    obs += t32(sig_np[:, :, None] * si.std_normal(tuple(obs.shape), 79))
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=128, generations=200, tournament_k=4, p_cross=0.85, p_mut=0.05, seed=0)
    stream = torch.cuda.current_stream(dev)
    res, ms = {}, {}
    for name, f in (("fill", fill), ("plain", None)):
        g.ga_invert(obs[:256], sig[:256], lines, grids, b, cfg, mu=mu[:256], fill=f)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        res[name] = g.ga_invert(obs, sig, lines, grids, b, cfg, mu=mu, fill=f)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms[name] = ev[0].elapsed_time(ev[1])
        print("fill: %s GA %.1f ms" % (name, ms[name]), file=sys.stderr, flush=True)

    def pct(x):
        return {"p50": float(np.percentile(x, 50)), "p90": float(np.percentile(x, 90))}

    strong = truth[:, 0] >= 500.0
    acc = {}
    for name in res:
        B = res[name]["params"][:, 0].cpu().numpy().astype(np.float64)
        acc[name] = {"abs_dB_G": pct(np.abs(B - truth[:, 0])),
                     "abs_dB_G_strong": pct(np.abs(B - truth[:, 0])[strong]),
                     "median_chi2": float(res[name]["chi2"].median().item())}
    da = np.abs(res["fill"]["alpha"].cpu().numpy().astype(np.float64) - alpha)
    acc["fill"]["abs_dalpha"] = pct(da)
    acc["fill"]["abs_dalpha_strong"] = pct(da[strong])
    L = sum(gr.n for gr in grids)
    fpe = flops_per_eval(list(zip(lines, grids))) + FLOP_FILL_PER_LAMBDA * L
    evals = npix * 128 * 201
    ga_s = ms["fill"] / 1e3
    out = {"metric": "pixel inversions/s with the magnetic fill fraction (GA, FP32)",
           "value": npix / ga_s, "unit": "pixels/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": ms["fill"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (truth from the priors, alpha U(0.25, 1), mu U(0.3, 1), "
                   "field-free stand-in profile, noise 1e-3 Ic)",
           "config": {"workload": "fill fraction: 2048 px x 2 lines x 128, pop 128, G 200, "
                                  "alpha in [0, 1] solved per individual", "npix": npix},
           "plain_ga_ms": ms["plain"], "accuracy": acc,
           "roofline": {"bound": "alu", "achieved": evals * fpe / ga_s / 1e12,
                        "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                        "frac": evals * fpe / ga_s / PEAK_FP32_VALU, "traffic": None,
                        "kernel": "k_ga_invert<float, fill>", "flop_per_eval": fpe,
                        "evals_per_launch": evals}}
    print(json.dumps(out), flush=True)


DISC_BLOCKS = 20          # contiguous scanline blocks of the full disc; one step = one block
DISC_GA = dict(pop=128, generations=150, k=4, p_mut=0.05, p_cross=0.85, seed=0,
               refine=REFINE_ITERS)


def _lineset(g, si, name="slit"):
    lines, grids = [], []
    for ln, n in si.line_set(name):
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
    return lines, grids


def _errors(params, truth):
    """p50/p90/p99 of |estimate - truth| per parameter (azimuth modulo 180
    deg; the angles only where B_truth >= 100 G)."""
    d = np.abs(params - truth)
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    strong = truth[:, 0] >= 100.0
    import synth_inputs as si
    out = {}
    for j, name in enumerate(si.PARAM_NAMES):
        x = d[strong, j] if name in ("incl", "azim") else d[:, j]
        out[name] = {q: float(np.percentile(x, int(q[1:]))) for q in ("p50", "p90", "p99")}
    return out


def disc_workload(args):
    """The full-disc map in DISC_BLOCKS scanline blocks (see the module
    docstring); returns the JSON record."""
    import torch
    import paper_1208_0302_amd as g
    from paper_1208_0302_amd import build as gbuild
    import synth_inputs as si

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    truth, mu_np, _ = si.full_disc(2048, seed=0, stride=1)
    npix = truth.shape[0]
    print("disc: %d on-disc pixels (%.1f s)" % (npix, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    lines, grids = _lineset(g, si)
    f64 = dict(dtype=torch.float64, device=dev)
    mu64 = torch.tensor(mu_np, **f64)
    obs64 = g.me_synth(torch.tensor(truth, **f64), lines, grids, mu=mu64)
    sig64 = torch.tensor(si.sigma_for(truth, mu=mu_np), **f64)
    obs32, sig32, mu32 = obs64.float(), sig64.float(), mu64.float()
    torch.cuda.synchronize()
    w = DISC_GA
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    edges = [npix * k // DISC_BLOCKS for k in range(DISC_BLOCKS + 1)]

    def launch(k):
        s0, s1 = edges[k], edges[k + 1]
        cfg = g.GAConfig(pop=w["pop"], generations=w["generations"], tournament_k=w["k"],
                         p_cross=w["p_cross"], p_mut=w["p_mut"], seed=w["seed"], pixel_base=s0)
        r = g.ga_invert(obs32[s0:s1], sig32[s0:s1], lines, grids, b, cfg, mu=mu32[s0:s1],
                        want_status=False)
        return r

    def refine(k, r):
        s0, s1 = edges[k], edges[k + 1]
        return g.me_refine_f64(obs64[s0:s1], sig64[s0:s1], lines, grids, b,
                               r["params"].double(), w["refine"], mu=mu64[s0:s1])

    for i in range(args.warmup):
        refine(i % DISC_BLOCKS, launch(i % DISC_BLOCKS))
        torch.cuda.synchronize()
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    ga_out, ref_out = {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done_px = 0
    for i in range(args.steps):
        k = i % DISC_BLOCKS
        ev[i][0].record(stream)
        r = launch(k)
        ev[i][1].record(stream)
        m = refine(k, r)
        ev[i][2].record(stream)
        ga_out[k], ref_out[k] = r["params"], m["params"]
        done_px += edges[k + 1] - edges[k]
        if i + 1 < args.steps:
            # progress line from the work itself: the previous step has ended
            ev[i][0].synchronize()
            print("step %d/%d (block %d) issued; step %d done" % (i + 1, args.steps, k, i),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ga_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    step_ms = np.array([e[0].elapsed_time(e[2]) for e in ev])
    print("steps done: ga kernel ms %s, step ms %s" % (np.round(ga_ms, 1).tolist(),
                                                       np.round(step_ms, 1).tolist()),
          file=sys.stderr, flush=True)
    blocks = sorted(ref_out)
    sel = np.concatenate([np.arange(edges[k], edges[k + 1]) for k in blocks])
    est = np.concatenate([ref_out[k].cpu().numpy() for k in blocks])
    est_ga = np.concatenate([ga_out[k].double().cpu().numpy() for k in blocks])
    acc = _errors(est, truth[sel])
    acc_ga = _errors(est_ga, truth[sel])
    dB = acc["B"]
    accuracy = {"p50_abs_dB_G": dB["p50"], "p90_abs_dB_G": dB["p90"], "p99_abs_dB_G": dB["p99"],
                "gate_p90_dB_le_10G": bool(dB["p90"] <= 10.0), "pixels": int(len(sel)),
                "per_parameter": acc, "ga_only": acc_ga,
                }
    lg = list(zip(lines, grids))
    fpe = flops_per_eval(lg)
    evals = np.array([(edges[(i % DISC_BLOCKS) + 1] - edges[i % DISC_BLOCKS])
                      * w["pop"] * (w["generations"] + 1) for i in range(args.steps)])
    achieved = float((evals * fpe).sum() / (ga_ms.sum() / 1e3))
    desc = ("full disc 2048^2: %d on-disc px in %d scanline blocks of %d-%d px x [%s], pop %d, "
            "G %d, k %d, p_mut %.2f, p_cross %.2f, FP32 GA + %d FP64 Levenberg-Marquardt "
            "iterations, noise-free observations"
            % (npix, DISC_BLOCKS, min(np.diff(edges)), max(np.diff(edges)),
               "; ".join("%.4f A (%d comp) x %d" % (ln.lambda0_A, ln.ncomp, gr.n)
                         for ln, gr in lg),
               w["pop"], w["generations"], w["k"], w["p_mut"], w["p_cross"], w["refine"]))
    out = {
        "metric": METRIC,
        "value": done_px / wall,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (smooth random parameter fields with 20-px correlation plus 1 % "
                "strong-field patches on a 2048^2 disc, mu from the disc position, noise-free "
                "observations from the FP64 forward model)",
        "config": {"workload": desc, "npix": npix, "blocks": DISC_BLOCKS,
                   "pixels_timed": done_px, "pop": w["pop"], "generations": w["generations"],
                   "seed": w["seed"], "refine_iterations": w["refine"]},
        "me_evals_per_s": float(evals.sum() / (ga_ms.sum() / 1e3)),
        "tile_ms_p50": float(np.percentile(step_ms, 50)),
        "tile_ms_p99": float(np.percentile(step_ms, 99)),
        "ga_kernel_ms": float(ga_ms.mean()),
        "refine_ms": float((step_ms - ga_ms).mean()),
        "accuracy": accuracy,
        "layout": gbuild.layout(),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU,
                     "traffic": disc_traffic(edges),
                     "kernel": "k_ga_invert<float>", "flop_per_eval": fpe,
                     "evals_per_launch": float(evals.mean())},
    }
    if not args.no_cpu_baseline:
        # a seeded sample of the disc's pixels; the oracle also checks the
        # benchmark's (device-made) observations of those pixels
        sample = np.sort(np.random.default_rng(1).choice(npix, 64, replace=False))
        out["cpu_baseline"] = cpu_baseline(dict(w, name="disc"), truth[sample], "slit",
                                           args.cpu_budget, mu=mu_np[sample],
                                           device_obs=obs64[torch.tensor(sample, device=dev)]
                                           .cpu().numpy())
    return out


def uncertainty_leg(g, w, obs, sig, obs64, sig64, lines, grids, b, cfg, popt, stream, reps=3):
    """Sec. 6 uncertainties of the refined pixels, after the timed steps: the
    initial steps from the final population of one more search (the same
    seed, so the same population), then me_uncertainty_f64 timed with HIP
    events on the launch stream."""
    import torch
    r = g.ga_invert(obs, sig, lines, grids, b, cfg, want_population=True)
    steps = g.ga_population_steps(r["genes"], r["fitness"], b, popt)
    u = g.me_uncertainty_f64(obs64, sig64, lines, grids, b, popt, steps)  # warm-up
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        u = g.me_uncertainty_f64(obs64, sig64, lines, grids, b, popt, steps)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    s = u["sigma"].cpu().numpy()
    fin = np.isfinite(s).all(axis=1)
    print("uncertainties done: %s ms" % np.round(ms, 3).tolist(), file=sys.stderr, flush=True)
    return {"kernel": "k_uncert_f64", "pixels": w["npix"], "ms": float(ms.mean()),
            "ms_min": float(ms.min()), "pixels_per_s": w["npix"] / (float(ms.mean()) / 1e3),
            "finite_fraction": float(fin.mean()),
            "median_sigma_B_G": float(np.median(s[fin, 0])) if fin.any() else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=DISC_BLOCKS)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="disc",
                    help="disc (default), slit, tiny, precision, serving, proposal, fill")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--uncertainty", action="store_true",
                    help="slit, tiny: after the timed steps, also time the Sec. 6 uncertainties "
                    "of the refined pixels (not part of a step)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--rate", type=float, default=2.0, help="serving: requests per second")
    ap.add_argument("--window", type=float, default=20.0, help="serving: arrival window [s]")
    ap.add_argument("--gens-per-step", type=int, default=10, help="serving: generations per launch")
    ap.add_argument("--tile-median", type=float, default=4096.0,
                    help="serving: median tile size in pixels (lognormal, sigma 1.2)")
    ap.add_argument("--max-resident-pixels", type=int, default=0,
                    help="serving: resident-pixel cap of the admission (0: memory budget only)")
    ap.add_argument("--disc-stride", type=int, default=16,
                    help="precision: keep every n-th on-disc pixel of the 2048^2 map")
    ap.add_argument("--batch", type=int, default=4096, help="proposal: training batch")
    ap.add_argument("--lr", type=float, default=2e-3, help="proposal: Adam learning rate")
    ap.add_argument("--heldout", type=int, default=16384, help="proposal: held-out pixels")
    ap.add_argument("--strategies", default="random,seeded,physics,polarity_box,prefit_box,"
                    "physics_in_box,sobol,sobol_restart," + ",".join(SEED_STRATEGIES) +
                    ",four_seeds,four_seeds_polarity,four_seeds_exact,four_seeds_exact_polarity",
                    help="proposal: initial-population strategies to compare")
    ap.add_argument("--chi2-target", type=float, default=1.2,
                    help="proposal: reduced chi-square target")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) so that "
                         "HBM byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: pixels are independent, so N GPUs would each invert "
              "their own share of the map. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    if args.workload == "serving":
        serving(args)
        return
    if args.workload == "proposal":
        proposal(args)
        return
    if args.workload == "precision":
        precision_study(args)
        return
    if args.workload == "disc":
        print(json.dumps(disc_workload(args)), flush=True)
        return
    if args.workload == "fill":
        fill_workload(args)
        return
    import paper_1208_0302_amd as g
    import synth_inputs as si

    w = workload(args.workload)
    dev = torch.device("cuda:0")
    dt = torch.float32 if w["dtype"] == "f32" else torch.float64
    specs = si.line_set(w["lines"])
    lines, grids = [], []
    for ln, n in specs:
        start, step = si.grid(ln, n)
        lines.append(g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]))
        grids.append(g.grid(start, step, n))
    truth = si.draw_truth(w["npix"], seed=w["seed"])
    # noise-free observations from the FP64 forward model (the search reads
    # them in its own precision)
    obs64 = g.me_synth(torch.tensor(truth, dtype=torch.float64, device=dev), lines, grids)
    sig64 = torch.tensor(si.sigma_for(truth), dtype=torch.float64, device=dev)
    obs, sig = obs64.to(dt).contiguous(), sig64.to(dt).contiguous()
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=w["pop"], generations=w["generations"], tournament_k=w["k"],
                     p_cross=w["p_cross"], p_mut=w["p_mut"], seed=w["seed"])
    torch.cuda.synchronize()

    def step():
        r = g.ga_invert(obs, sig, lines, grids, b, cfg)
        m = g.me_refine_f64(obs64 if dt == torch.float32 else obs, sig64, lines, grids, b,
                            r["params"].double().contiguous(), w["refine"])
        return r, m

    for i in range(args.warmup):
        step()
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        res = g.ga_invert(obs, sig, lines, grids, b, cfg)
        ev[i][1].record(stream)
        ref = g.me_refine_f64(obs64 if dt == torch.float32 else obs, sig64, lines, grids, b,
                              res["params"].double().contiguous(), w["refine"])
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ga_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    step_ms = np.array([e[0].elapsed_time(e[2]) for e in ev])
    print("steps done: ga kernel ms %s, step ms %s" % (np.round(ga_ms, 3).tolist(),
                                                       np.round(step_ms, 3).tolist()),
          file=sys.stderr, flush=True)

    # accuracy on the noise-free truth (the gate: p90 |dB| <= 10 G)
    def acc_of(params):
        dB = np.abs(params[:, 0] - truth[:, 0])
        return {"p50_abs_dB_G": float(np.percentile(dB, 50)),
                "p90_abs_dB_G": float(np.percentile(dB, 90)),
                "p99_abs_dB_G": float(np.percentile(dB, 99))}
    acc = acc_of(ref["params"].cpu().numpy())
    acc["gate_p90_dB_le_10G"] = bool(acc["p90_abs_dB_G"] <= 10.0)
    acc["median_chi2"] = float(ref["chi2"].median().item())
    acc["ga_only"] = acc_of(res["params"].double().cpu().numpy())

    npix = w["npix"]
    evals = npix * w["pop"] * (w["generations"] + 1)
    fpe = flops_per_eval(list(zip(lines, grids)))
    flop_launch = evals * fpe
    mean_s = float(ga_ms.mean()) / 1e3
    achieved = flop_launch / mean_s
    peak = PEAK_FP32_VALU if dt == torch.float32 else PEAK_FP64_VALU
    out = {
        "metric": METRIC,
        "value": npix * args.steps / wall,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["dtype"],
        "data": "synthetic (truth from the priors, noise-free observations from the forward model)",
        "config": {"workload": describe(w, list(zip(lines, grids))), "npix": npix,
                   "pop": w["pop"], "generations": w["generations"], "seed": w["seed"],
                   "refine_iterations": w["refine"]},
        "me_evals_per_s": evals / mean_s,
        "tile_ms_p50": float(np.percentile(step_ms, 50)),
        "tile_ms_p99": float(np.percentile(step_ms, 99)),
        "ga_kernel_ms": float(ga_ms.mean()),
        "refine_ms": float((step_ms - ga_ms).mean()),
        "accuracy": acc,
        "layout": __import__("paper_1208_0302_amd.build", fromlist=["layout"]).layout(),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": (measured_traffic(TRAFFIC_SLIT_BYTES)
                                 if w["name"] == "slit" and dt == torch.float32 else None),
                     "kernel": "k_ga_invert<%s>" % ("float" if dt == torch.float32 else "double"),
                     "flop_per_eval": fpe, "evals_per_launch": evals},
    }
    if args.uncertainty:
        out["uncertainty"] = uncertainty_leg(g, w, obs, sig, obs64, sig64, lines, grids, b, cfg,
                                             ref["params"], stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, truth, w["lines"], args.cpu_budget,
                                           device_obs=obs64.cpu().numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
