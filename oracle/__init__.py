"""FP64 CPU oracle for Milne-Eddington genetic-algorithm Stokes inversion.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference the HIP path
is checked against (Harker & Mighell, "A GPU-Computing Approach to Solar Stokes
Profile Inversion": Sec. 3 genetic algorithm, Sec. 4.2 16-bit genes, Sec. 5
Milne-Eddington synthesis and chi-square).  Only ``tests/``, the smoke check and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
HIP library and never imports it.

The C sources next to this file are compiled with gcc (OpenMP over pixels) into
``liboracle.so``; ``build()`` does that and ``lib()`` builds on first use when
the shared object is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("oracle_me.c", "oracle_ga.c", "oracle_lm.c",
                                          "oracle_fill.c", "oracle_unc.c")]
_LOCK = threading.Lock()
_LIB = None

NPAR = 9
MAXCOMP = 64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -fopenmp into liboracle.so."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-ffp-contract=off",
           "-D_GNU_SOURCE", "-o", tmp] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class Line(C.Structure):
    _fields_ = [
        ("lambda0", C.c_double),
        ("ncomp", C.c_int32),
        ("q", C.c_int32 * MAXCOMP),
        ("shift", C.c_double * MAXCOMP),
        ("strength", C.c_double * MAXCOMP),
        ("start", C.c_double),
        ("step", C.c_double),
        ("nlam", C.c_int32),
    ]


MAXLINES = 8


class FillLine(C.Structure):
    _fields_ = [("depth", C.c_double * 4), ("width", C.c_double * 4), ("damp", C.c_double * 4)]


class Fill(C.Structure):
    """Fill fraction (Sec. 5.2): alpha range and, per line, the cubic-in-mu
    coefficients of the field-free profile's depth, width [A] and damping."""
    _fields_ = [("alpha_lo", C.c_double), ("alpha_hi", C.c_double),
                ("line", FillLine * MAXLINES)]


def make_fill(alpha_lo, alpha_hi, depth, width, damp) -> Fill:
    """depth, width, damp: [nlines, 4] cubic coefficients (mu^0 .. mu^3)."""
    f = Fill()
    f.alpha_lo, f.alpha_hi = float(alpha_lo), float(alpha_hi)
    for l in range(len(depth)):
        for k in range(4):
            f.line[l].depth[k] = float(depth[l][k])
            f.line[l].width[k] = float(width[l][k])
            f.line[l].damp[k] = float(damp[l][k])
    return f


_dp = C.POINTER(C.c_double)
_u16p = C.POINTER(C.c_uint16)
_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)
_linep = C.POINTER(Line)
OBJECTIVE = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)


def lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            newest_src = max(os.path.getmtime(s) for s in _SRC + [os.path.join(_HERE, "oracle.h")])
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < newest_src:
                build()
            L = C.CDLL(_SO)
            L.oracle_faddeeva.argtypes = [C.c_double, C.c_double, _dp, _dp]
            L.oracle_lande_ls.argtypes = [C.c_double] * 3
            L.oracle_lande_ls.restype = C.c_double
            L.oracle_wigner3j.argtypes = [C.c_double] * 6
            L.oracle_wigner3j.restype = C.c_double
            L.oracle_zeeman.argtypes = [C.c_double] * 4 + [_i32p, _dp, _dp, C.c_int]
            L.oracle_zeeman.restype = C.c_int
            L.oracle_me_synth.argtypes = [_dp, C.c_int64, _linep, C.c_int, _dp, _dp]
            L.oracle_me_synth_lin.argtypes = [_dp, _dp, C.c_double, _linep, C.c_int, _dp]
            L.oracle_chi2.argtypes = [_dp, C.c_int64, C.c_int, _linep, C.c_int, _dp, _dp, _dp, _dp]
            L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
            L.oracle_rng_word.argtypes = [C.c_uint64] + [C.c_uint32] * 5
            L.oracle_rng_word.restype = C.c_uint32
            L.oracle_decode.argtypes = [_u16p, _dp, _dp, _dp]
            L.oracle_ga_init.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int, C.c_int, _dp,
                                         _dp, _dp, C.c_int, _u16p]
            L.oracle_sobol_polys.argtypes = [_u32p, C.c_int]
            L.oracle_sobol_polys.restype = C.c_int
            L.oracle_sobol_point.argtypes = [C.c_uint32, _u32p]
            L.oracle_ga_restart.argtypes = [_u16p, _dp, C.c_int, C.c_uint64, C.c_uint32, C.c_int,
                                            C.c_int, _u16p, _i32p]
            L.oracle_ga_step.argtypes = [_u16p, _dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                         C.c_uint64, C.c_uint32, C.c_uint32,
                                         _u16p, _i32p, _i32p, _u16p, _i32p]
            L.oracle_ga_step.restype = C.c_int
            L.oracle_ga_invert.argtypes = [_dp, _dp, _dp, C.c_int64, _linep, C.c_int, _dp, _dp,
                                           _dp, C.POINTER(Fill), _dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                           C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int,
                                           _dp, C.c_int, C.c_int, _dp, _dp, _i32p, _u16p, _dp]
            L.oracle_ga_invert.restype = C.c_int
            L.oracle_lm_refine.argtypes = [_dp, _dp, _dp, C.c_int64, _linep, C.c_int, _dp, _dp,
                                           _dp, C.c_int, _dp, _dp, _i32p]
            L.oracle_lm_refine.restype = C.c_int
            L.oracle_lm_fit.argtypes = [_dp, _dp, _dp, C.c_int64, _linep, C.c_int, _dp, _dp,
                                        _dp, C.c_int, C.c_uint32, _dp, _dp, _i32p]
            L.oracle_lm_fit.restype = C.c_int
            L.oracle_lm_fit_fill.argtypes = [_dp, _dp, _dp, C.c_int64, _linep, C.c_int, _dp,
                                             _dp, C.POINTER(Fill), _dp, _dp, C.c_int,
                                             C.c_uint32, _dp, _dp, _dp, _i32p]
            L.oracle_lm_fit_fill.restype = C.c_int
            L.oracle_uncertainty.argtypes = [_dp, _dp, _dp, C.c_int64, _linep, C.c_int, _dp,
                                             _dp, _dp, _dp, C.c_uint32, _dp, _dp, _dp, _dp]
            L.oracle_uncertainty.restype = C.c_int
            L.oracle_population_steps.argtypes = [_u16p, _dp, C.c_int64, C.c_int, _dp, _dp,
                                                  _dp, _dp]
            L.oracle_population_steps.restype = C.c_int
            L.oracle_sec6_hessian.argtypes = [OBJECTIVE, C.c_void_p, C.c_int, _dp, _dp, _i32p,
                                              _dp, _dp]
            L.oracle_sec6_hessian.restype = C.c_int
            L.oracle_sec6_sigmas.argtypes = [_dp, _i32p, C.c_double, C.c_int, _dp]
            L.oracle_sec6_sigmas.restype = C.c_int
            L.oracle_fill_profile.argtypes = [_linep, C.POINTER(FillLine), C.c_double,
                                              C.c_double, _dp]
            L.oracle_fill_profile.restype = C.c_int
            L.oracle_me_synth_fill.argtypes = [_dp, _dp, C.c_int64, _linep, C.c_int, _dp,
                                               C.POINTER(Fill), _dp]
            L.oracle_me_synth_fill.restype = C.c_int
            L.oracle_chi2_fill.argtypes = [_dp, C.c_int64, C.c_int, _linep, C.c_int, _dp, _dp,
                                           _dp, C.POINTER(Fill), _dp, _dp]
            L.oracle_chi2_fill.restype = None
            L.oracle_num_threads.restype = C.c_int
            _LIB = L
    return _LIB


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- #
# special functions and atomic data

def faddeeva(x, y):
    """w(x + i y) elementwise (numpy broadcasting); complex128."""
    x, y = np.broadcast_arrays(np.asarray(x, np.float64), np.asarray(y, np.float64))
    out = np.empty(x.shape, np.complex128)
    re, im = C.c_double(), C.c_double()
    L = lib()
    for idx in np.ndindex(x.shape):
        L.oracle_faddeeva(float(x[idx]), float(y[idx]), C.byref(re), C.byref(im))
        out[idx] = complex(re.value, im.value)
    return out


def lande_ls(S, Lq, J):
    return lib().oracle_lande_ls(float(S), float(Lq), float(J))


def wigner3j(j1, j2, j3, m1, m2, m3):
    return lib().oracle_wigner3j(*(float(v) for v in (j1, j2, j3, m1, m2, m3)))


def zeeman(Jl, gl, Ju, gu):
    """Components (q, shift, strength) of the J_l -> J_u transition."""
    q = np.zeros(MAXCOMP, np.int32)
    s = np.zeros(MAXCOMP, np.float64)
    st = np.zeros(MAXCOMP, np.float64)
    n = lib().oracle_zeeman(float(Jl), float(gl), float(Ju), float(gu),
                            _ptr(q, _i32p), _ptr(s, _dp), _ptr(st, _dp), MAXCOMP)
    if n < 0:
        raise ValueError("invalid transition")
    return q[:n].copy(), s[:n].copy(), st[:n].copy()


def make_line(lambda0, Jl, gl, Ju, gu, start, step, nlam) -> Line:
    q, s, st = zeeman(Jl, gl, Ju, gu)
    ln = Line()
    ln.lambda0 = float(lambda0)
    ln.ncomp = len(q)
    for i in range(len(q)):
        ln.q[i] = int(q[i])
        ln.shift[i] = float(s[i])
        ln.strength[i] = float(st[i])
    ln.start = float(start)
    ln.step = float(step)
    ln.nlam = int(nlam)
    return ln


def _lines_array(lines):
    arr = (Line * len(lines))(*lines)
    return arr, C.cast(arr, _linep)


def total_samples(lines):
    return sum(int(l.nlam) for l in lines)


# --------------------------------------------------------------------------- #
# forward model and merit function

def me_synth(params, lines, mu=None):
    """Stokes [n, 4, L] for params [n, 9] (FP64)."""
    p = _f64(params).reshape(-1, NPAR)
    n = p.shape[0]
    L = total_samples(lines)
    out = np.empty((n, 4, L), np.float64)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (n,)))
    lib().oracle_me_synth(_ptr(p, _dp), n, lp, len(lines),
                          None if m is None else _ptr(m, _dp), _ptr(out, _dp))
    return out


def me_synth_lin(params0, params, lines, mu=1.0):
    """Stokes [4, L] of params [9] with every component's Faddeeva value taken
    to first order about its value at params0 [9] (oracle_me_synth_lin)."""
    p0 = np.ascontiguousarray(_f64(params0).reshape(NPAR))
    p = np.ascontiguousarray(_f64(params).reshape(NPAR))
    out = np.empty((4, total_samples(lines)), np.float64)
    arr, lp = _lines_array(lines)
    lib().oracle_me_synth_lin(_ptr(p0, _dp), _ptr(p, _dp), float(mu), lp, len(lines),
                              _ptr(out, _dp))
    return out


def chi2(params, obs, sigma, lines, mu=None):
    """chi-square [npix, pop] of params [npix, pop, 9] against obs [npix, 4, L]."""
    p = _f64(params)
    npix, pop = p.shape[0], p.shape[1]
    o = _f64(obs)
    s = _f64(sigma)
    out = np.empty((npix, pop), np.float64)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    lib().oracle_chi2(_ptr(p, _dp), npix, pop, lp, len(lines), _ptr(o, _dp), _ptr(s, _dp),
                      None if m is None else _ptr(m, _dp), _ptr(out, _dp))
    return out


# --------------------------------------------------------------------------- #
# random stream and genetic operators

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def rng_word(seed, pixel, gen, indiv, purpose, n):
    return lib().oracle_rng_word(int(seed), int(pixel), int(gen), int(indiv), int(purpose), int(n))


def decode(genes, lo, hi):
    g = np.ascontiguousarray(genes, np.uint16).reshape(-1, NPAR)
    lo = _f64(lo)
    hi = _f64(hi)
    out = np.empty(g.shape, np.float64)
    for i in range(g.shape[0]):
        lib().oracle_decode(_ptr(g[i], _u16p), _ptr(lo, _dp), _ptr(hi, _dp), _ptr(out[i], _dp))
    return out.reshape(np.shape(genes))


def ga_init(seed, pixel, pop, n_seeded=0, jitter=0, seed_params=None, lo=None, hi=None,
            init_mode=0):
    """Generation 0 of one pixel; the first n_seeded individuals encode the
    first guesses seed_params [9] or [S, 9] inside the box [lo, hi] (Sec.
    5.5; individual i takes guess i mod S); the rest are uniform random
    (init_mode 0) or shifted Sobol points (1, Sec. 5.6)."""
    g = np.empty((pop, NPAR), np.uint16)
    sp = lo_ = hi_ = None
    S = 1
    if n_seeded > 0:
        sp, lo_, hi_ = _f64(seed_params).reshape(-1, NPAR), _f64(lo), _f64(hi)
        S = sp.shape[0]
    lib().oracle_ga_init(int(seed), int(pixel), int(pop), int(n_seeded), int(jitter), int(S),
                         None if sp is None else _ptr(sp, _dp),
                         None if lo_ is None else _ptr(lo_, _dp),
                         None if hi_ is None else _ptr(hi_, _dp), int(init_mode), _ptr(g, _u16p))
    return g


def sobol_polys(n):
    out = np.zeros(n, np.uint32)
    got = lib().oracle_sobol_polys(_ptr(out, _u32p), int(n))
    return out[:got]


def sobol_point(n):
    out = np.empty(NPAR, np.uint32)
    lib().oracle_sobol_point(int(n), _ptr(out, _u32p))
    return out


def ga_restart(genes_in, fitness, seed, pixel, t, restart_every):
    """Restart after generation t; returns (genes, replaced flags)."""
    g = np.ascontiguousarray(genes_in, np.uint16)
    pop = g.shape[0]
    f = _f64(fitness)
    out = np.empty_like(g)
    rep = np.empty(pop, np.int32)
    lib().oracle_ga_restart(_ptr(g, _u16p), _ptr(f, _dp), pop, int(seed), int(pixel), int(t),
                            int(restart_every), _ptr(out, _u16p), _ptr(rep, _i32p))
    return out, rep.astype(bool)


def ga_step(genes_in, fitness, k, p_cross, p_mut, seed, pixel, gen):
    """One generation; returns dict(genes, parents, xpoint, masks, elite)."""
    g = np.ascontiguousarray(genes_in, np.uint16)
    pop = g.shape[0]
    f = _f64(fitness)
    out = np.empty_like(g)
    parents = np.empty((pop, 2), np.int32)
    xp = np.empty(pop, np.int32)
    masks = np.empty_like(g)
    e = C.c_int32()
    rc = lib().oracle_ga_step(_ptr(g, _u16p), _ptr(f, _dp), pop, int(k), float(p_cross),
                              float(p_mut), int(seed), int(pixel), int(gen), _ptr(out, _u16p),
                              _ptr(parents, _i32p), _ptr(xp, _i32p), _ptr(masks, _u16p),
                              C.byref(e))
    if rc != 0:
        raise ValueError("oracle_ga_step rejected its arguments")
    return dict(genes=out, parents=parents, xpoint=xp, masks=masks, elite=int(e.value))


def ga_invert(obs, sigma, lines, lo, hi, pop, generations, k, p_cross, p_mut, seed,
              mu=None, pixel_base=0, want_population=False, n_seeded=0, seed_jitter=0,
              seed_params=None, init_mode=0, restart_every=0, pixel_box=None, fill=None):
    """Algorithm 1 for npix pixels; seed_params [npix, 9] or [npix, S, 9]
    (S first guesses per pixel); pixel_box [npix, 2, 9] (lo row, hi row)
    gives each pixel its own search box (status 3 where it is invalid); fill
    (a Fill) makes the fitness the chi-square at the best fill fraction and
    adds 'alpha' [npix] to the result (status 4 where the field-free profile
    is invalid)."""
    o = _f64(obs)
    s = _f64(sigma)
    npix = o.shape[0]
    lo = _f64(lo)
    hi = _f64(hi)
    pb = None if pixel_box is None else _f64(pixel_box).reshape(npix, 2, NPAR)
    ba = np.empty(npix, np.float64)
    bp = np.empty((npix, NPAR), np.float64)
    bc = np.empty(npix, np.float64)
    st = np.empty(npix, np.int32)
    fg = np.empty((npix, pop, NPAR), np.uint16) if want_population else None
    ff = np.empty((npix, pop), np.float64) if want_population else None
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    sp = None if n_seeded == 0 else _f64(seed_params).reshape(npix, -1, NPAR)
    S = 1 if sp is None else sp.shape[1]
    rc = lib().oracle_ga_invert(
        _ptr(o, _dp), _ptr(s, _dp), None if m is None else _ptr(m, _dp), npix, lp, len(lines),
        _ptr(lo, _dp), _ptr(hi, _dp), None if pb is None else _ptr(pb, _dp),
        None if fill is None else C.byref(fill), None if fill is None else _ptr(ba, _dp), int(pop),
        int(generations), int(k), float(p_cross),
        float(p_mut), int(seed), int(pixel_base), int(n_seeded), int(seed_jitter), int(S),
        None if sp is None else _ptr(sp, _dp), int(init_mode), int(restart_every), _ptr(bp, _dp), _ptr(bc, _dp), _ptr(st, _i32p),
        None if fg is None else _ptr(fg, _u16p), None if ff is None else _ptr(ff, _dp))
    if rc != 0:
        raise ValueError("oracle_ga_invert rejected its arguments")
    res = dict(params=bp, chi2=bc, status=st)
    if fill is not None:
        res["alpha"] = ba
    if want_population:
        res.update(genes=fg, fitness=ff)
    return res


def fill_profile(line, fill_line, mu, vlos):
    """Normalised field-free profile N [nlam] of one line (oracle_fill.c)."""
    out = np.empty(line.nlam, np.float64)
    if lib().oracle_fill_profile(C.byref(line), C.byref(fill_line), float(mu), float(vlos),
                                 _ptr(out, _dp)) != 0:
        raise ValueError("field-free profile invalid at this mu")
    return out


def me_synth_fill(params, alpha, lines, fill, mu=None):
    """alpha M + (1 - alpha) I_c N e: Stokes [n, 4, L] for params [n, 9] and
    alpha [n] (FP64)."""
    p = _f64(params).reshape(-1, NPAR)
    n = p.shape[0]
    a = _f64(np.broadcast_to(alpha, (n,)))
    L = sum(ln.nlam for ln in lines)
    out = np.empty((n, 4, L), np.float64)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (n,)))
    lib().oracle_me_synth_fill(_ptr(p, _dp), _ptr(a, _dp), n, lp, len(lines),
                               None if m is None else _ptr(m, _dp), C.byref(fill), _ptr(out, _dp))
    return out


def chi2_fill(params, obs, sigma, lines, fill, mu=None):
    """(chi-square, best alpha) [npix, pop] of params [npix, pop, 9] (nu = 4L - 10)."""
    p = _f64(params)
    npix, pop = p.shape[0], p.shape[1]
    o = _f64(obs)
    s = _f64(sigma)
    c = np.empty((npix, pop), np.float64)
    a = np.empty((npix, pop), np.float64)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    lib().oracle_chi2_fill(_ptr(p, _dp), npix, pop, lp, len(lines), _ptr(o, _dp), _ptr(s, _dp),
                           None if m is None else _ptr(m, _dp), C.byref(fill), _ptr(c, _dp),
                           _ptr(a, _dp))
    return c, a


def lm_refine(obs, sigma, lines, lo, hi, params_in, iterations, mu=None, free_mask=0x1FF):
    """FP64 Levenberg-Marquardt refinement; returns dict(params, chi2, iters).
    Only the parameters in free_mask (bit j = parameter j) are adjusted."""
    o = _f64(obs)
    s = _f64(sigma)
    npix = o.shape[0]
    p0 = _f64(params_in).reshape(npix, NPAR)
    lo = _f64(lo)
    hi = _f64(hi)
    po = np.empty((npix, NPAR), np.float64)
    co = np.empty(npix, np.float64)
    it = np.empty(npix, np.int32)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    rc = lib().oracle_lm_fit(_ptr(o, _dp), _ptr(s, _dp), None if m is None else _ptr(m, _dp),
                             npix, lp, len(lines), _ptr(lo, _dp), _ptr(hi, _dp),
                             _ptr(p0, _dp), int(iterations), int(free_mask), _ptr(po, _dp),
                             _ptr(co, _dp), _ptr(it, _i32p))
    if rc != 0:
        raise ValueError("oracle_lm_fit rejected its arguments")
    return dict(params=po, chi2=co, iters=it)


def lm_refine_fill(obs, sigma, lines, lo, hi, fill, params_in, alpha_in, iterations, mu=None,
                   free_mask=0x3FF):
    """FP64 Levenberg-Marquardt refinement of the fill-fraction model (Sec.
    5.2) over the nine parameters and alpha (bit 9 of free_mask); returns
    dict(params, alpha, chi2, iters) with nu = 4L - 10."""
    o = _f64(obs)
    s = _f64(sigma)
    npix = o.shape[0]
    p0 = _f64(params_in).reshape(npix, NPAR)
    a0 = _f64(np.broadcast_to(alpha_in, (npix,)))
    lo = _f64(lo)
    hi = _f64(hi)
    po = np.empty((npix, NPAR), np.float64)
    ao = np.empty(npix, np.float64)
    co = np.empty(npix, np.float64)
    it = np.empty(npix, np.int32)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    rc = lib().oracle_lm_fit_fill(_ptr(o, _dp), _ptr(s, _dp), None if m is None else _ptr(m, _dp),
                                  npix, lp, len(lines), _ptr(lo, _dp), _ptr(hi, _dp),
                                  C.byref(fill), _ptr(p0, _dp), _ptr(a0, _dp), int(iterations),
                                  int(free_mask), _ptr(po, _dp), _ptr(ao, _dp), _ptr(co, _dp),
                                  _ptr(it, _i32p))
    if rc != 0:
        raise ValueError("oracle_lm_fit_fill rejected its arguments")
    return dict(params=po, alpha=ao, chi2=co, iters=it)


def uncertainty(obs, sigma, lines, lo, hi, p_opt, steps, mu=None, free_mask=0x1FF):
    """Sec. 6 uncertainties at p_opt [npix, 9] from initial steps [npix, 9];
    returns dict(sigma, hess, hess_err, steps) (see oracle_unc.c)."""
    o = _f64(obs)
    s = _f64(sigma)
    npix = o.shape[0]
    q = _f64(p_opt).reshape(npix, NPAR)
    h = _f64(steps).reshape(npix, NPAR)
    lo = _f64(lo)
    hi = _f64(hi)
    sg = np.empty((npix, NPAR), np.float64)
    H = np.empty((npix, NPAR, NPAR), np.float64)
    He = np.empty((npix, NPAR, NPAR), np.float64)
    hu = np.empty((npix, NPAR), np.float64)
    arr, lp = _lines_array(lines)
    m = None if mu is None else _f64(np.broadcast_to(mu, (npix,)))
    rc = lib().oracle_uncertainty(_ptr(o, _dp), _ptr(s, _dp), None if m is None else _ptr(m, _dp),
                                  npix, lp, len(lines), _ptr(lo, _dp), _ptr(hi, _dp),
                                  _ptr(q, _dp), _ptr(h, _dp), int(free_mask), _ptr(sg, _dp),
                                  _ptr(H, _dp), _ptr(He, _dp), _ptr(hu, _dp))
    if rc != 0:
        raise ValueError("oracle_uncertainty rejected its arguments")
    return dict(sigma=sg, hess=H, hess_err=He, steps=hu)


def population_steps(genes, fitness, lo, hi, p_opt):
    """Sec. 6 initial steps [npix, 9] from a final population genes [npix,
    pop, 9] (uint16), fitness [npix, pop]."""
    g = np.ascontiguousarray(genes, np.uint16)
    npix, pop = g.shape[0], g.shape[1]
    f = _f64(fitness).reshape(npix, pop)
    q = _f64(p_opt).reshape(npix, NPAR)
    out = np.empty((npix, NPAR), np.float64)
    rc = lib().oracle_population_steps(_ptr(g, _u16p), _ptr(f, _dp), npix, pop,
                                       _ptr(_f64(lo), _dp), _ptr(_f64(hi), _dp), _ptr(q, _dp),
                                       _ptr(out, _dp))
    if rc != 0:
        raise ValueError("oracle_population_steps rejected its arguments")
    return out


def sec6_hessian(f, p, h, active=None):
    """The Sec. 6 Hessian (same tableaux) of a Python objective f(p) of n <= 9
    variables at p with initial steps h; returns (H, error estimates)."""
    n = len(p)
    q = _f64(p)
    hh = _f64(h)
    act = np.ones(n, np.int32) if active is None else np.ascontiguousarray(active, np.int32)
    H = np.empty((n, n), np.float64)
    He = np.empty((n, n), np.float64)

    def cb(ptr, ctx):
        return float(f(np.ctypeslib.as_array(ptr, shape=(n,)).copy()))
    fn = OBJECTIVE(cb)
    rc = lib().oracle_sec6_hessian(fn, None, n, _ptr(q, _dp), _ptr(hh, _dp), _ptr(act, _i32p),
                                   _ptr(H, _dp), _ptr(He, _dp))
    if rc != 0:
        raise ValueError("oracle_sec6_hessian rejected its arguments")
    return H, He


def sec6_sigmas(H, active, chi2, M):
    """sigma_j = sqrt([H^-1]_jj chi2 / M) over the active parameters of a 9 x 9 H."""
    Hm = _f64(H).reshape(NPAR, NPAR)
    act = np.ascontiguousarray(active, np.int32)
    out = np.empty(NPAR, np.float64)
    rc = lib().oracle_sec6_sigmas(_ptr(Hm, _dp), _ptr(act, _i32p), float(chi2), int(M),
                                  _ptr(out, _dp))
    if rc != 0:
        raise ValueError("oracle_sec6_sigmas rejected its arguments")
    return out


PREFIT_FREE = 0x1F8   # v_los, Doppler width, damping, eta0, S0, S1


def prefit(obs, sigma, lines, lo, hi, params_in, iterations, mu=None):
    """Non-magnetic pre-fit (Sec. 5.3): the Levenberg-Marquardt fit of the
    model with B held at 0 (so neither field angle matters and Q = U = V =
    0), adjusting v_los, the Doppler width, damping, eta0, S0 and S1 from
    params_in; the box must contain B = 0."""
    lo = _f64(lo)
    hi = _f64(hi)
    if not lo[0] <= 0.0 <= hi[0]:
        raise ValueError("the box must contain B = 0")
    p0 = _f64(params_in).reshape(-1, NPAR).copy()
    p0[:, 0] = 0.0
    return lm_refine(obs, sigma, lines, lo, hi, p0, iterations, mu=mu, free_mask=PREFIT_FREE)


def num_threads():
    return lib().oracle_num_threads()
