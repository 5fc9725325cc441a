"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/genesis.h declares, its host-only line data agree with the
oracle's Zeeman pattern, and invalid arguments fail before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1208_0302_amd as g
import synth_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genesis.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = g.lib()
    declared = _declared()
    assert len(declared) >= 35
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(g.EXPORTED) == declared
    assert L.genesis_abi_version() == g.ABI_VERSION == 5


def test_binding_structs_match_the_library():
    # the binding refuses to load when a layout differs (a stale field list
    # would hand the device garbage pointers); check the sizes directly too
    L = g.lib()
    for which, (name, struct) in enumerate(g.STRUCTS):
        assert L.genesis_struct_size(which) == C.sizeof(struct), name
    assert L.genesis_struct_size(len(g.STRUCTS)) == 0
    assert g.GaConfigC.pixel_bounds.offset == 64 and C.sizeof(g.GaConfigC) == 72


def _sorted_components(q, s, st):
    return sorted(zip(np.asarray(q).tolist(), np.round(s, 12).tolist(), np.round(st, 12).tolist()))


@pytest.mark.parametrize("Jl,Ju", [(2, 2), (1, 0), (0, 1), (1, 1), (1, 2), (2, 1), (3, 4),
                                   (1.5, 2.5), (2.5, 1.5), (0.5, 0.5), (4, 3), (3.5, 3.5)])
def test_host_zeeman_matches_oracle(Jl, Ju):
    rng = np.random.default_rng(int(10 * Jl + Ju))
    gl, gu = rng.uniform(0.5, 2.5, 2)
    ln = g.line_from_terms(6000.0, Jl, gl, Ju, gu)
    q, s, st = oracle.zeeman(Jl, gl, Ju, gu)
    got = _sorted_components(ln.q[:ln.ncomp], np.array(ln.shift[:ln.ncomp]),
                             np.array(ln.strength[:ln.ncomp]))
    assert got == _sorted_components(q, s, st)


def test_table1_lines_host():
    for line, n in ((si.FE6301, 12), (si.FE6302, 3)):
        ln = g.line_from_terms(line["lambda0"], line["Jl"], line["gl"], line["Ju"], line["gu"])
        assert ln.ncomp == n


def test_triplet():
    ln = g.line_triplet(6302.5, 2.5)
    assert ln.ncomp == 3
    assert list(ln.q[:3]) == [-1, 0, 1]
    assert list(ln.shift[:3]) == [-2.5, 0.0, 2.5]


def test_invalid_arguments_fail_before_device_work():
    L = g.lib()
    ln = g.line_from_terms(6302.5017, 1, 2.5, 0, 0)
    la = (g.MeLine * 1)(ln)
    ga = (g.MeGrid * 1)(g.grid(6302.1, 0.008, 100))
    # nlines out of range
    assert L.me_synth(None, 4, la, ga, 0, None, None, None) == g.ME_EINVAL
    assert b"nlines" in L.me_last_error()
    # NULL arrays with n > 0
    assert L.me_synth(None, 4, la, ga, 1, None, None, None) == g.ME_EINVAL
    # n = 0 is a no-op
    assert L.me_synth(None, 0, la, ga, 1, None, None, None) == g.ME_OK
    # not a dipole transition
    out = g.MeLine()
    assert L.me_line_from_terms(6300.0, 2.0, 1.0, 0.0, 1.0, C.byref(out)) == g.ME_EINVAL
    # bad GA configurations
    for kw in (dict(pop=1), dict(pop=2000), dict(tournament_k=9), dict(tournament_k=0),
               dict(p_cross=1.5), dict(p_mut=-0.1), dict(generations=-1)):
        cfg = g.GAConfig(**{**dict(pop=16, tournament_k=4), **kw}).c()
        assert L.ga_init(4, C.byref(cfg), None, None, None) == g.ME_EINVAL
    # bad seeding: more seeded slots than the population, jitter out of range,
    # seeded slots without first guesses or without a search box
    for kw in (dict(n_seeded=17), dict(n_seeded=-1), dict(seed_jitter=40000)):
        cfg = g.GAConfig(**{**dict(pop=16), **kw}).c()
        assert L.ga_init(4, C.byref(cfg), None, None, None) == g.ME_EINVAL
    cfg = g.GAConfig(pop=16, n_seeded=4).c()
    assert L.ga_init(4, C.byref(cfg), None, None, None) == g.ME_EINVAL
    assert b"seed_params" in L.me_last_error()
    cfg.seed_params = 256          # never dereferenced: the missing box fails first
    assert L.ga_init(4, C.byref(cfg), None, None, None) == g.ME_EINVAL
    # synthesis precision: unknown value; FP16 only for the FP32 entry point and
    # damping bounds within [0, 1]
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    cfg = g.GAConfig(pop=16, synth_precision=2).c()
    assert L.ga_init(4, C.byref(cfg), None, None, None) == g.ME_EINVAL
    cfg = g.GAConfig(pop=16, synth_precision=g.SYNTH_FP16).c()
    assert L.ga_invert_f64(None, None, None, 3, la, ga, 1, C.byref(b), C.byref(cfg), None, None,
                           None, None, None, None, 0, None) == g.ME_EINVAL
    wide = g.bounds(si.PRIOR_LO, np.where(np.arange(9) == 5, 1.5, si.PRIOR_HI))
    assert L.ga_invert(None, None, None, 3, la, ga, 1, C.byref(wide), C.byref(cfg), None, None,
                       None, None, None, None, 0, None) == g.ME_EINVAL
    assert b"FP16" in L.me_last_error()
    cfg = g.GAConfig(pop=16).c()
    assert L.ga_step(None, None, 2, C.byref(cfg), 0, None, None, None, None, None,
                     None) == g.ME_EINVAL      # generation 0 is not a step
    b = g.bounds(si.PRIOR_LO, si.PRIOR_HI)
    bad = g.bounds(si.PRIOR_HI, si.PRIOR_LO)
    assert L.ga_decode(None, 3, C.byref(bad), None, None) == g.ME_EINVAL
    assert L.ga_invert(None, None, None, 3, la, ga, 1, C.byref(b), C.byref(cfg), None, None,
                       None, None, None, None, 0, None) == g.ME_EINVAL
    # too few samples for nu = 4L - 9 > 0
    ga2 = (g.MeGrid * 1)(g.grid(6302.1, 0.008, 2))
    assert L.ga_invert(None, None, None, 3, la, ga2, 1, C.byref(b), C.byref(cfg), None, None,
                       None, None, None, None, 0, None) == g.ME_EINVAL
    # LDS limit: 4 lines x 1100 samples do not fit
    la4 = (g.MeLine * 4)(ln, ln, ln, ln)
    ga4 = (g.MeGrid * 4)(*([g.grid(6302.1, 0.001, 1100)] * 4))
    assert L.ga_invert(None, None, None, 3, la4, ga4, 4, C.byref(b), C.byref(cfg), None, None,
                       None, None, None, None, 0, None) == g.ME_ENOMEM
    assert L.ga_workspace_bytes(100, C.byref(cfg)) == 0
    # inverse-max weights: a negative or non-finite floor, no grids, an empty grid
    assert L.me_invmax_sigma(None, 3, ga, 1, -1.0, None, None) == g.ME_EINVAL
    assert L.me_invmax_sigma_f64(None, 3, ga, 1, float("nan"), None, None) == g.ME_EINVAL
    assert L.me_invmax_sigma(None, 3, ga, 0, 1e-3, None, None) == g.ME_EINVAL
    assert L.me_invmax_sigma(None, 3, (g.MeGrid * 1)(g.grid(6302.1, 0.008, 0)), 1, 1e-3, None,
                             None) == g.ME_EINVAL
    assert L.me_invmax_sigma(None, 3, ga, 1, 1e-3, None, None) == g.ME_EINVAL   # NULL arrays
    assert L.me_invmax_sigma(None, 0, ga, 1, 1e-3, None, None) == g.ME_OK       # empty


def test_product_and_oracle_are_independent():
    pkg = os.path.join(ROOT, "paper_1208_0302_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", text, flags=re.M), f
                assert "oracle.h" not in text and "liboracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1208_0302_amd" not in text and "genesis.h" not in text, f
