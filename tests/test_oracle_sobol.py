"""Pins of the oracle's Sobol points and restarts (Sec. 5.6).

The primitive polynomials are pinned by the number-theoretic count of
primitive polynomials of each degree, phi(2^d - 1)/d, and by the textbook list
of small ones; the points by the closed form of dimension 0 (bit reversal),
the textbook start of dimension 1, and the net properties every Sobol sequence
has (each one-dimensional projection of the first 2^m points is a (0, m, 1)
net; dimensions 0 and 1 form a (0, m, 2) net); restarts by which individuals
they replace, and the whole loop by its composition from the operators."""
import math

import numpy as np

import oracle
import synth_inputs as si


def _phi(n):
    r, m, p = n, n, 2
    while p * p <= m:
        if m % p == 0:
            while m % p == 0:
                m //= p
            r -= r // p
        p += 1
    if m > 1:
        r -= r // m
    return r


def test_primitive_polynomials():
    polys = oracle.sobol_polys(60)
    assert list(polys[:8]) == [0b11, 0b111, 0b1011, 0b1101, 0b10011, 0b11001, 0b100101,
                               0b101001]
    degs = np.array([int(p).bit_length() - 1 for p in polys])
    for d in range(1, 7):
        assert (degs == d).sum() == _phi(2 ** d - 1) // d, d
    # increasing within a degree, degrees non-decreasing
    assert np.all(np.diff(polys.astype(np.int64)) > 0)


def test_dimension_zero_is_bit_reversal():
    for n in (0, 1, 2, 3, 5, 12, 1000, 123456, 2 ** 31 + 7):
        rev = int("{:032b}".format(n)[::-1], 2)
        assert oracle.sobol_point(n)[0] == rev


def test_dimension_one_textbook_start():
    x = [oracle.sobol_point(n)[1] / 2.0 ** 32 for n in range(1, 8)]
    assert x == [0.5, 0.75, 0.25, 0.625, 0.125, 0.375, 0.875]


def test_one_dimensional_nets():
    for m in (1, 4, 7, 10):
        pts = np.array([oracle.sobol_point(n) for n in range(2 ** m)], np.uint64)
        for d in range(9):
            cells = pts[:, d] >> np.uint64(32 - m)
            assert len(np.unique(cells)) == 2 ** m, (m, d)


def test_two_dimensional_net_of_dimensions_zero_and_one():
    m = 8
    pts = np.array([oracle.sobol_point(n)[:2] for n in range(2 ** m)], np.uint64)
    for k in range(m + 1):
        a = pts[:, 0] >> np.uint64(32 - k) if k else np.zeros(2 ** m, np.uint64)
        b = pts[:, 1] >> np.uint64(32 - (m - k)) if m - k else np.zeros(2 ** m, np.uint64)
        boxes = a * np.uint64(2 ** (m - k)) + b
        assert len(np.unique(boxes)) == 2 ** m, k


def test_sobol_population_is_stratified_per_gene():
    # the per-pixel digital shift permutes the cells, so the first 64 points
    # still put one gene into each of the 64 equal cells of [0, 65535]
    g = oracle.ga_init(5, 17, 64, init_mode=1)
    for j in range(9):
        assert len(np.unique(g[:, j] >> 10)) == 64
    # different pixels get different (shifted) populations
    assert not np.array_equal(g, oracle.ga_init(5, 18, 64, init_mode=1))
    # seeded slots still take precedence
    gs = oracle.ga_init(5, 17, 64, n_seeded=3, jitter=0, seed_params=si.PRIOR_HI,
                        lo=si.PRIOR_LO, hi=si.PRIOR_HI, init_mode=1)
    assert np.all(gs[:3] == 65535) and np.array_equal(gs[3:], g[3:])


def test_restart_replaces_the_worst_half():
    rng = np.random.default_rng(0)
    pop = 20
    genes = si.random_genes(1, pop, 3)[0]
    fit = rng.permutation(pop).astype(float)
    fit[4] = fit[9]                       # a tie: the lower index ranks first
    fit[7] = np.nan                       # NaN ranks last
    out, rep = oracle.ga_restart(genes, fit, seed=11, pixel=2, t=10, restart_every=5)
    order = sorted(range(pop), key=lambda i: (np.inf if np.isnan(fit[i]) else fit[i], i))
    worst = order[pop - pop // 2:]
    assert set(np.nonzero(rep)[0]) == set(worst)
    assert np.array_equal(out[~rep], genes[~rep])
    # rank pop - nrep + q takes Sobol point pop + (t/R - 1) nrep + q
    shift = np.array([oracle.rng_word(11, 2, 0, 0, 4, j) for j in range(9)], np.uint32)
    for q, i in enumerate(worst):
        pt = oracle.sobol_point(pop + (10 // 5 - 1) * (pop // 2) + q)
        assert np.array_equal(out[i], ((pt ^ shift) >> 16).astype(np.uint16))
    assert 7 in worst


def _lines():
    return [oracle.make_line(l["lambda0"], l["Jl"], l["gl"], l["Ju"], l["gu"], *si.grid(l, n), n)
            for l, n in si.line_set("tiny")]


def test_loop_with_restarts_is_the_composition_of_its_operators():
    lines = _lines()
    truth = si.draw_truth(2, 4)
    obs = oracle.me_synth(truth, lines)
    sig = si.sigma_for(truth)
    lo, hi = si.PRIOR_LO, si.PRIOR_HI
    pop, G, R, k, pc, pm, seed = 16, 9, 3, 4, 0.85, 0.05, 21
    res = oracle.ga_invert(obs, sig, lines, lo, hi, pop, G, k, pc, pm, seed, init_mode=1,
                           restart_every=R, want_population=True)
    for p in range(2):
        g = oracle.ga_init(seed, p, pop, init_mode=1)
        f = oracle.chi2(oracle.decode(g, lo, hi)[None], obs[p:p + 1], sig[p:p + 1], lines)[0]
        for t in range(1, G + 1):
            if (t - 1) > 0 and (t - 1) % R == 0:
                g, rep = oracle.ga_restart(g, f, seed, p, t - 1, R)
                f = oracle.chi2(oracle.decode(g, lo, hi)[None], obs[p:p + 1], sig[p:p + 1],
                                lines)[0]
            g = oracle.ga_step(g, f, k, pc, pm, seed, p, t)["genes"]
            f = oracle.chi2(oracle.decode(g, lo, hi)[None], obs[p:p + 1], sig[p:p + 1], lines)[0]
        assert np.array_equal(res["genes"][p], g)
        assert np.array_equal(res["fitness"][p], f)
    # restarts beyond the last generation change nothing
    a = oracle.ga_invert(obs, sig, lines, lo, hi, pop, G, k, pc, pm, seed, restart_every=G,
                         want_population=True)
    b = oracle.ga_invert(obs, sig, lines, lo, hi, pop, G, k, pc, pm, seed, want_population=True)
    assert np.array_equal(a["genes"], b["genes"])
    assert math.isfinite(res["chi2"][0])
