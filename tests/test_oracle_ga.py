"""Pins of the oracle's genetic operators (Sec. 3, Algorithm 1; Sec. 4.2).

The operators are stochastic, so they are pinned by the laws their readings
imply: the closed-form win probability of a tournament of k distinct
contestants, uniform crossover points, the per-bit mutation probabilities, the
exact reconstruction of every child from its parents, and the properties of the
whole loop (elitism, determinism, checkpoint/resume).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth_inputs as si

POP = 64
K = 4
PC = 0.85
PM = 0.05


def _steps(ncalls, pop=POP, k=K, pc=PC, pm=PM, fitness=None, seed=99):
    out = []
    for c in range(ncalls):
        genes = si.random_genes(1, pop, seed + c)[0]
        f = fitness if fitness is not None else np.random.default_rng(c).permutation(pop).astype(float)
        out.append((genes, f, oracle.ga_step(genes, f, k, pc, pm, seed, pixel=c, gen=1 + c % 7)))
    return out


def test_tournament_rank_law():
    # distinct fitness: rank r (1 = best) wins with probability C(n-r, k-1)/C(n, k)
    n = POP
    counts = np.zeros(n, np.int64)
    for genes, f, r in _steps(1500):
        rank = np.argsort(np.argsort(f))        # 0 = best
        pairs = r["parents"][1::2]              # one row per pair
        for a, b in pairs:
            counts[rank[a]] += 1
            counts[rank[b]] += 1
    total = counts.sum()
    p = np.array([math.comb(n - r, K - 1) / math.comb(n, K) for r in range(1, n + 1)])
    assert abs(p.sum() - 1) < 1e-12
    exp = p * total
    keep = exp >= 20
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    assert stats.chisquare(obs, ex).pvalue > 1e-4
    # the worst k-1 individuals can never win a tournament of k distinct contestants
    assert counts[n - K + 1:].sum() == 0


def test_tournament_ties_and_nan():
    # all equal: the lowest index among the contestants wins, so the winner
    # follows the same law with index order as rank
    n = 16
    counts = np.zeros(n, np.int64)
    for genes, f, r in _steps(3000, pop=n, fitness=np.ones(n)):
        for a, b in r["parents"][1::2]:
            counts[a] += 1
            counts[b] += 1
    p = np.array([math.comb(n - r, K - 1) / math.comb(n, K) for r in range(1, n + 1)])
    keep = p * counts.sum() >= 20
    assert stats.chisquare(counts[keep], p[keep] * counts.sum() * counts[keep].sum()
                           / (p[keep] * counts.sum()).sum()).pvalue > 1e-4
    assert counts[~keep].sum() <= 100 and counts[n - K + 1:].sum() == 0
    # NaN is +infinity: a single finite individual wins every tournament it
    # enters, and is the elite
    f = np.full(n, np.nan)
    f[5] = 3.0
    for genes, _, r in _steps(200, pop=n, fitness=f):
        assert r["elite"] == 5
    genes = si.random_genes(1, n, 4)[0]
    r = oracle.ga_step(genes, f, K, PC, PM, 1, 0, 1)
    assert r["elite"] == 5


def test_crossover_frequency_and_points():
    xs = []
    npairs = 0
    for genes, f, r in _steps(1500):
        x = r["xpoint"][1::2]
        npairs += len(x)
        xs.extend(x[x > 0].tolist())
    xs = np.array(xs)
    # crossover happens with probability p_c
    z = (len(xs) - PC * npairs) / math.sqrt(npairs * PC * (1 - PC))
    assert abs(z) < 4.5
    # the point is uniform on [1, 143]
    assert xs.min() >= 1 and xs.max() <= 143
    counts = np.bincount(xs, minlength=144)[1:]
    assert stats.chisquare(counts).pvalue > 1e-4


def test_mutation_bit_frequencies():
    ones = np.zeros(16, np.int64)
    trials = 0
    for genes, f, r in _steps(600):
        m = r["masks"][1:]                       # children only
        trials += m.size
        for k in range(16):
            ones[k] += int(np.count_nonzero(m & (1 << (15 - k))))
    for k in range(16):
        pk = 2 * PM * (k + 1) / 17
        z = (ones[k] - pk * trials) / math.sqrt(trials * pk * (1 - pk))
        assert abs(z) < 4.5, (k, z)
    # more-significant bits flip less often (Sec. 3)
    assert np.all(np.diff(ones) > 0)


def _cross(a, b, x):
    bits_a = np.unpackbits(a.astype(">u2").view(np.uint8))
    bits_b = np.unpackbits(b.astype(">u2").view(np.uint8))
    c1 = np.concatenate([bits_a[:x], bits_b[x:]])
    c2 = np.concatenate([bits_b[:x], bits_a[x:]])
    return (np.packbits(c1).view(">u2").astype(np.uint16),
            np.packbits(c2).view(">u2").astype(np.uint16))


def test_children_reconstruct_from_parents():
    for genes, f, r in _steps(60, pop=33) + _steps(60, pop=32):
        pop = genes.shape[0]
        e = r["elite"]
        assert e == int(np.lexsort((np.arange(pop), f))[0])
        assert np.array_equal(r["genes"][0], genes[e])
        for c in range(1, pop):
            a, b = r["parents"][c]
            x = r["xpoint"][c]
            c1, c2 = _cross(genes[a], genes[b], x) if x else (genes[a], genes[b])
            child = c1 if (c - 1) % 2 == 0 else c2
            assert np.array_equal(r["genes"][c], child ^ r["masks"][c])


def test_step_rejects_bad_arguments():
    genes = si.random_genes(1, 8, 0)[0]
    f = np.arange(8.0)
    with pytest.raises(ValueError):
        oracle.ga_step(genes, f, 9, PC, PM, 0, 0, 1)        # k > pop
    with pytest.raises(ValueError):
        oracle.ga_step(genes, f, 2, 1.5, PM, 0, 0, 1)       # p_cross > 1
    with pytest.raises(ValueError):
        oracle.ga_step(genes, f, 2, PC, PM, 0, 0, 0)        # generation 0 is the initial one


# --------------------------------------------------------------------------- #
# whole loop

def _tiny_problem(npix=3, seed=0, noise=False):
    line, n = si.line_set("tiny")[0]
    start, step = si.grid(line, n)
    ln = oracle.make_line(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"],
                          start, step, n)
    truth = si.draw_truth(npix, seed)
    obs = oracle.me_synth(truth, [ln])
    sig = si.sigma_for(truth)
    if noise:
        obs = obs + sig[:, :, None] * si.std_normal(obs.shape, seed)
    return [ln], truth, obs, sig


def test_loop_determinism_and_resume():
    lines, truth, obs, sig = _tiny_problem()
    kw = dict(lo=si.PRIOR_LO, hi=si.PRIOR_HI, pop=16, k=4, p_cross=PC, p_mut=PM, seed=7)
    a = oracle.ga_invert(obs, sig, lines, generations=4, want_population=True, **kw)
    b = oracle.ga_invert(obs, sig, lines, generations=4, want_population=True, **kw)
    assert np.array_equal(a["genes"], b["genes"]) and np.array_equal(a["chi2"], b["chi2"])
    # a run to generation 8 equals a run to 4 resumed for 4 more generations
    full = oracle.ga_invert(obs, sig, lines, generations=8, want_population=True, **kw)
    for p in range(obs.shape[0]):
        g, f = a["genes"][p], a["fitness"][p]
        for t in range(5, 9):
            g = oracle.ga_step(g, f, 4, PC, PM, 7, p, t)["genes"]
            par = oracle.decode(g, si.PRIOR_LO, si.PRIOR_HI)
            f = oracle.chi2(par[None], obs[p:p + 1], sig[p:p + 1], lines)[0]
        assert np.array_equal(g, full["genes"][p])
        assert np.array_equal(f, full["fitness"][p])
    # elitism: the best chi-square never increases
    assert np.all(full["chi2"] <= a["chi2"])


def test_loop_initial_population_matches_init():
    lines, truth, obs, sig = _tiny_problem(npix=2)
    r = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, pop=8, generations=0, k=2,
                         p_cross=PC, p_mut=PM, seed=3, pixel_base=10, want_population=True)
    for p in range(2):
        assert np.array_equal(r["genes"][p], oracle.ga_init(3, 10 + p, 8))


def test_loop_status_codes():
    lines, truth, obs, sig = _tiny_problem(npix=3)
    obs = obs.copy()
    sig = sig.copy()
    obs[1, 2, 5] = np.nan
    sig[2, 3] = 0.0
    r = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, pop=8, generations=1, k=2,
                         p_cross=PC, p_mut=PM, seed=3)
    assert list(r["status"]) == [0, 1, 2]
    assert np.isfinite(r["chi2"][0]) and np.isnan(r["chi2"][1:]).all()


def test_loop_without_variation_only_reselects_generation_zero():
    # with neither crossover nor mutation the loop can create no genotype:
    # every final individual is one of generation 0, carries that genotype's
    # chi-square, and the best is generation 0's best (kept by elitism)
    lines, truth, obs, sig = _tiny_problem(npix=3, seed=4, noise=True)
    kw = dict(lo=si.PRIOR_LO, hi=si.PRIOR_HI, pop=16, k=3, p_cross=0.0, p_mut=0.0, seed=5,
              want_population=True)
    r0 = oracle.ga_invert(obs, sig, lines, generations=0, **kw)
    r = oracle.ga_invert(obs, sig, lines, generations=6, **kw)
    for p in range(3):
        first = {tuple(g): f for g, f in zip(r0["genes"][p].tolist(), r0["fitness"][p])}
        for g, f in zip(r["genes"][p].tolist(), r["fitness"][p]):
            assert tuple(g) in first and f == first[tuple(g)]
        assert r["chi2"][p] == r0["fitness"][p].min()
        assert np.array_equal(r["genes"][p][0], r0["genes"][p][np.argmin(r0["fitness"][p])])


@pytest.mark.parametrize("pc", [0.0, 1.0])
def test_loop_tournament_over_everyone_breeds_only_the_best(pc):
    # a tournament of the whole population always picks generation 0's best,
    # and crossing it with itself gives itself: one generation turns the
    # population into copies of that genotype
    lines, truth, obs, sig = _tiny_problem(npix=2, seed=6, noise=True)
    kw = dict(lo=si.PRIOR_LO, hi=si.PRIOR_HI, pop=8, k=8, p_cross=pc, p_mut=0.0, seed=9,
              want_population=True)
    r0 = oracle.ga_invert(obs, sig, lines, generations=0, **kw)
    r = oracle.ga_invert(obs, sig, lines, generations=1, **kw)
    for p in range(2):
        best = r0["genes"][p][np.argmin(r0["fitness"][p])]
        assert np.array_equal(r["genes"][p], np.broadcast_to(best, r["genes"][p].shape))
        assert np.all(r["fitness"][p] == r0["fitness"][p].min())


@pytest.mark.slow
def test_loop_converges_on_noise_free_truth():
    # the general trajectory has no closed form; the whole loop must still
    # drive chi-square towards zero on noise-free synthetic truth
    lines, truth, obs, sig = _tiny_problem(npix=8, seed=2)
    r0 = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, pop=64, generations=0, k=4,
                          p_cross=PC, p_mut=PM, seed=0)
    r = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, pop=64, generations=60, k=4,
                         p_cross=PC, p_mut=PM, seed=0)
    ratio = r["chi2"] / r0["chi2"]
    assert np.all(ratio < 0.5) and np.median(ratio) < 0.02


# ---- seeding of generation 0 with first guesses (Sec. 5.5) -------------------

def test_seeded_init_encodes_and_jitters():
    lo, hi = si.PRIOR_LO, si.PRIOR_HI
    guess = si.draw_uniform_box(1, 5)[0]
    pop, ns, jit = 64, 40, 3
    g = oracle.ga_init(7, 11, pop, n_seeded=ns, jitter=jit, seed_params=guess, lo=lo, hi=hi)
    # individual 0 decodes to the nearest code of the guess: within half a step
    dec = oracle.decode(g[0], lo, hi)
    assert np.all(np.abs(dec - guess) <= 0.5 * (hi - lo) / 65535 * (1 + 1e-12))
    # the jittered copies stay within +-jit codes and use every offset
    d = g[1:ns].astype(int) - g[0].astype(int)
    assert np.abs(d).max() <= jit
    assert set(np.unique(d)) == set(range(-jit, jit + 1))
    # offsets are near-uniform over 2 jit + 1 values (39 x 9 draws)
    counts = np.array([(d == v).sum() for v in range(-jit, jit + 1)])
    assert stats.chisquare(counts).pvalue > 1e-4
    # the unseeded tail is the plain random population, unchanged by seeding
    assert np.array_equal(g[ns:], oracle.ga_init(7, 11, pop)[ns:])
    # no seeds: the plain population
    assert np.array_equal(oracle.ga_init(7, 11, pop, n_seeded=0, jitter=jit),
                          oracle.ga_init(7, 11, pop))


def test_seeded_init_clamps_to_box():
    lo, hi = si.PRIOR_LO, si.PRIOR_HI
    guess = np.where(np.arange(9) % 2 == 0, lo - 5.0, hi + 5.0)
    g = oracle.ga_init(1, 0, 8, n_seeded=8, jitter=100, seed_params=guess, lo=lo, hi=hi)
    want = np.where(np.arange(9) % 2 == 0, 0, 65535)
    assert np.array_equal(g[0], want)
    # jitter never leaves [0, 65535]
    assert g.min() >= 0 and g.max() <= 65535
    assert np.all(np.abs(g[1:].astype(int) - want) <= 100)
    # exact box corners encode exactly
    g = oracle.ga_init(1, 0, 2, n_seeded=1, seed_params=hi, lo=lo, hi=hi)
    assert np.all(g[0] == 65535)
    g = oracle.ga_init(1, 0, 2, n_seeded=1, seed_params=lo, lo=lo, hi=hi)
    assert np.all(g[0] == 0)


def test_seeded_inversion_starts_at_the_guess():
    # a perfect first guess makes generation 0 already near-optimal: with no
    # generations the best chi-square is that of the truth's nearest code,
    # far below the random population's best
    lines = [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
             for l, n in si.line_set("tiny")]
    truth = si.draw_truth(4, 21)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    obs = obs + sig[:, :, None] * si.std_normal(obs.shape, 21)
    kw = dict(pop=32, generations=0, k=4, p_cross=0.85, p_mut=0.05, seed=3)
    r0 = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, **kw)
    r1 = oracle.ga_invert(obs, sig, lines, si.PRIOR_LO, si.PRIOR_HI, n_seeded=8, seed_jitter=50,
                          seed_params=truth, **kw)
    nu = 4 * 100 - 9
    assert np.all(r1["chi2"] < 2.0)            # reduced chi-square ~ 1 at the truth
    assert np.all(r0["chi2"] > 10.0 * r1["chi2"])
    # the elite of generation 0 is the exactly encoded guess or a jittered copy
    codes = np.array([oracle.ga_init(3, p, 32, 8, 50, truth[p], si.PRIOR_LO, si.PRIOR_HI)
                      for p in range(4)])
    direct = oracle.chi2(oracle.decode(codes[:, :1], si.PRIOR_LO, si.PRIOR_HI), obs, sig,
                         lines)[:, 0]
    assert np.all(r1["chi2"] <= direct * (1 + 1e-12))
    assert nu > 0


def test_seeded_init_nan_leaves_a_parameter_unseeded():
    lo, hi = si.PRIOR_LO, si.PRIOR_HI
    guess = si.draw_uniform_box(1, 6)[0]
    guess[[4, 5, 6]] = np.nan
    for mode in (0, 1):
        g = oracle.ga_init(2, 9, 32, n_seeded=10, jitter=20, seed_params=guess, lo=lo, hi=hi,
                           init_mode=mode)
        plain = oracle.ga_init(2, 9, 32, init_mode=mode)
        assert np.array_equal(g[:, [4, 5, 6]], plain[:, [4, 5, 6]])
        assert np.array_equal(g[10:], plain[10:])
        full = oracle.ga_init(2, 9, 32, n_seeded=10, jitter=20,
                              seed_params=np.nan_to_num(guess), lo=lo, hi=hi, init_mode=mode)
        keep = [0, 1, 2, 3, 7, 8]
        assert np.array_equal(g[:, keep], full[:, keep])


def _gen0(npix=300, pop=128, seed=11):
    return np.stack([oracle.ga_init(seed, p, pop) for p in range(npix)])   # [npix, pop, 9]


def test_initial_population_genes_are_uniform():
    # Algorithm 1 starts from a random population: every gene is a uniform
    # 16-bit value, so each of its bits is a fair coin and its top six bits
    # fall evenly into 64 bins; the decoded parameter is uniform on [lo, hi]
    g = _gen0().reshape(-1, si.NPAR).astype(np.int64)
    n = g.shape[0]
    tests = 0
    pmin = 1.0
    for j in range(si.NPAR):
        counts = np.bincount(g[:, j] >> 10, minlength=64)
        pmin = min(pmin, stats.chisquare(counts).pvalue)
        for b in range(16):
            ones = int(((g[:, j] >> b) & 1).sum())
            pmin = min(pmin, stats.binomtest(ones, n, 0.5).pvalue)
        tests += 17
    assert pmin > 1e-4 / tests, pmin
    par = oracle.decode(g[:4000].astype(np.uint16), si.PRIOR_LO, si.PRIOR_HI)
    for j in range(si.NPAR):
        u = (par[:, j] - si.PRIOR_LO[j]) / (si.PRIOR_HI[j] - si.PRIOR_LO[j])
        assert stats.kstest(u, "uniform").pvalue > 1e-4 / si.NPAR


def test_initial_population_genes_are_pairwise_independent():
    # independent draws: the joint 8 x 8 histogram of the top three bits of any
    # two genes of one individual, of one gene in neighbouring individuals and
    # in neighbouring pixels is the product of the marginals (a dropped index
    # in the random stream's counter would repeat values and fail here)
    g = _gen0().astype(np.int64) >> 13                    # [npix, pop, 9] in 0..7
    pairs = []
    for a in range(si.NPAR):
        for b in range(a + 1, si.NPAR):
            pairs.append((g[:, :, a].ravel(), g[:, :, b].ravel()))
    for j in range(si.NPAR):
        pairs.append((g[:, :-1, j].ravel(), g[:, 1:, j].ravel()))
        pairs.append((g[:-1, :, j].ravel(), g[1:, :, j].ravel()))
    pmin = 1.0
    for x, y in pairs:
        table = np.zeros((8, 8), np.int64)
        np.add.at(table, (x, y), 1)
        pmin = min(pmin, stats.chi2_contingency(table, correction=False).pvalue)
    assert pmin > 1e-4 / len(pairs), pmin
    # no two individuals of a pixel and no two pixels share a genotype
    full = _gen0(npix=50, pop=128)
    rows = {bytes(r) for r in full.reshape(-1, si.NPAR).astype(np.uint16)}
    assert len(rows) == 50 * 128


def test_initial_population_depends_on_seed_and_pixel_only():
    a = oracle.ga_init(5, 17, 64)
    assert np.array_equal(a, oracle.ga_init(5, 17, 64))
    assert not np.array_equal(a, oracle.ga_init(6, 17, 64))
    assert not np.array_equal(a, oracle.ga_init(5, 18, 64))
    # a larger population extends the smaller one (individual i's genes
    # depend on i, not on the population size)
    assert np.array_equal(oracle.ga_init(5, 17, 128)[:64], a)
