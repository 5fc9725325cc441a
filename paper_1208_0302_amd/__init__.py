"""Python binding of libgenesis_hip.so (C ABI in include/genesis.h).

Genetic-algorithm Milne-Eddington inversion of solar Stokes profiles on
MI355X (gfx950), after Harker & Mighell, "A GPU-Computing Approach to Solar
Stokes Profile Inversion".  This module only marshals arguments: every step of
the computation runs in the library's HIP kernels.  PyTorch supplies device
memory and the current stream.  There is no CPU fallback: if the shared object
is missing, loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import threading
from typing import Optional, Sequence

import torch

from . import build as _build

NPAR = 9
MAX_COMP = 32
MAX_LINES = 4
MAX_POP = 1024
MAX_K = 8

ME_OK, ME_EINVAL, ME_ENOMEM, ME_EHIP, ME_EBUSY = 0, -1, -2, -3, -4


class GenesisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("genesis error %d: %s" % (code, msg))
        self.code = code


class MeLine(C.Structure):
    _fields_ = [("lambda0_A", C.c_double), ("ncomp", C.c_int32),
                ("q", C.c_int32 * MAX_COMP), ("shift", C.c_double * MAX_COMP),
                ("strength", C.c_double * MAX_COMP)]


class MeGrid(C.Structure):
    _fields_ = [("start_A", C.c_double), ("step_A", C.c_double), ("n", C.c_int32)]


class MeBounds(C.Structure):
    _fields_ = [("lo", C.c_double * NPAR), ("hi", C.c_double * NPAR)]


class MeFill(C.Structure):
    """Fill fraction (Sec. 5.2): alpha range and per line the cubic-in-mu
    coefficients of the field-free profile's depth, width [A] and damping."""
    _fields_ = [("alpha_lo", C.c_double), ("alpha_hi", C.c_double),
                ("depth", (C.c_double * 4) * MAX_LINES), ("width", (C.c_double * 4) * MAX_LINES),
                ("damp", (C.c_double * 4) * MAX_LINES)]


def fill(alpha_lo, alpha_hi, depth, width, damp) -> MeFill:
    """MeFill from [nlines, 4] coefficient arrays (mu^0 .. mu^3)."""
    f = MeFill()
    f.alpha_lo, f.alpha_hi = float(alpha_lo), float(alpha_hi)
    for l in range(len(depth)):
        for k in range(4):
            f.depth[l][k] = float(depth[l][k])
            f.width[l][k] = float(width[l][k])
            f.damp[l][k] = float(damp[l][k])
    return f


SYNTH_NATIVE = 0
SYNTH_FP16 = 1


class GaConfigC(C.Structure):
    _fields_ = [("pop", C.c_int32), ("generations", C.c_int32), ("tournament_k", C.c_int32),
                ("n_seeded", C.c_int32), ("p_cross", C.c_float), ("p_mut", C.c_float),
                ("seed", C.c_uint64), ("pixel_base", C.c_uint32), ("seed_jitter", C.c_int32),
                ("seed_params", C.c_void_p), ("synth_precision", C.c_int32),
                ("init_mode", C.c_int32), ("restart_every", C.c_int32),
                ("seed_sets", C.c_int32), ("pixel_bounds", C.c_void_p)]


@dataclasses.dataclass
class GAConfig:
    """Genetic-algorithm settings (Sec. 3, Algorithm 1)."""
    pop: int = 128
    generations: int = 200
    tournament_k: int = 4
    p_cross: float = 0.85
    p_mut: float = 0.05
    seed: int = 0
    pixel_base: int = 0
    n_seeded: int = 0
    seed_jitter: int = 0
    seed_params: Optional[torch.Tensor] = None   # [npix, 9] or [npix, S, 9] float32 device tensor
    synth_precision: int = 0                     # SYNTH_NATIVE or SYNTH_FP16
    init_mode: int = 0                           # 0 uniform random, 1 Sobol
    restart_every: int = 0                       # 0: no restarts
    pixel_bounds: Optional[torch.Tensor] = None  # [npix, 2, 9] float32 per-pixel boxes

    def c(self, npix: Optional[int] = None) -> GaConfigC:
        """The C struct; with npix, the per-pixel arrays' shapes are checked."""
        cfg = GaConfigC()
        cfg.pop = self.pop
        cfg.generations = self.generations
        cfg.tournament_k = self.tournament_k
        cfg.p_cross = self.p_cross
        cfg.p_mut = self.p_mut
        cfg.seed = self.seed
        cfg.pixel_base = self.pixel_base
        cfg.n_seeded = self.n_seeded
        cfg.seed_jitter = self.seed_jitter
        cfg.synth_precision = self.synth_precision
        cfg.init_mode = self.init_mode
        cfg.restart_every = self.restart_every
        if self.seed_params is not None:
            sp = self.seed_params
            S = 1 if sp.dim() == 2 else sp.shape[1]
            _dev(sp, torch.float32, "seed_params",
                 None if npix is None else ((npix, NPAR) if sp.dim() == 2 else (npix, S, NPAR)))
            cfg.seed_params = sp.data_ptr()
            cfg.seed_sets = S
        if self.pixel_bounds is not None:
            _dev(self.pixel_bounds, torch.float32, "pixel_bounds",
                 None if npix is None else (npix, 2, NPAR))
            cfg.pixel_bounds = self.pixel_bounds.data_ptr()
        return cfg


_LOCK = threading.Lock()
_LIB = None

_vp = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32
_lp = C.POINTER(MeLine)
_gp = C.POINTER(MeGrid)
_bp = C.POINTER(MeBounds)
_cp = C.POINTER(GaConfigC)

_SIGS = {
    "me_last_error": ([], C.c_char_p),
    "genesis_abi_version": ([], C.c_int),
    "genesis_struct_size": ([_i32], C.c_size_t),
    "me_line_from_terms": ([C.c_double] * 5 + [_lp], C.c_int),
    "me_line_triplet": ([C.c_double, C.c_double, _lp], C.c_int),
    "me_synth": ([_vp, _i64, _lp, _gp, _i32, _vp, _vp, _vp], C.c_int),
    "me_synth_f64": ([_vp, _i64, _lp, _gp, _i32, _vp, _vp, _vp], C.c_int),
    "me_synth_f16": ([_vp, _i64, _lp, _gp, _i32, _vp, _vp, _vp], C.c_int),
    "me_chi2": ([_vp, _i64, _i32, _vp, _vp, _vp, _lp, _gp, _i32, _vp, _vp], C.c_int),
    "me_chi2_f64": ([_vp, _i64, _i32, _vp, _vp, _vp, _lp, _gp, _i32, _vp, _vp], C.c_int),
    "ga_init": ([_i64, _cp, _bp, _vp, _vp], C.c_int),
    "ga_restart": ([_vp, _vp, _i64, _cp, _i32, _vp, _vp], C.c_int),
    "ga_restart_f64": ([_vp, _vp, _i64, _cp, _i32, _vp, _vp], C.c_int),
    "ga_decode": ([_vp, _i64, _bp, _vp, _vp], C.c_int),
    "ga_evaluate": ([_vp, _i64, _i32, _bp, _vp, _vp, _vp, _lp, _gp, _i32, _vp, _vp], C.c_int),
    "ga_evaluate_f64": ([_vp, _i64, _i32, _bp, _vp, _vp, _vp, _lp, _gp, _i32, _vp, _vp],
                        C.c_int),
    "ga_step": ([_vp, _vp, _i64, _cp, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ga_step_f64": ([_vp, _vp, _i64, _cp, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ga_workspace_bytes": ([_i64, _cp], C.c_size_t),
    "ga_invert": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp, _vp, _vp, _vp, _vp, _vp, _vp,
                   C.c_size_t, _vp], C.c_int),
    "ga_invert_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp, _vp, _vp, _vp, _vp, _vp,
                       _vp, C.c_size_t, _vp], C.c_int),
    "me_refine_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, _i32, _vp, _vp, _vp, _vp],
                      C.c_int),
    "me_refine_fill_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, C.POINTER(MeFill), _vp,
                            _vp, _i32, C.c_uint32, _vp, _vp, _vp, _vp, _vp], _i32),
    "me_uncertainty_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, _vp, C.c_uint32, _vp,
                            _vp, _vp, _vp, _vp], C.c_int),
    "ga_population_steps": ([_vp, _vp, _i64, _i32, _bp, _vp, _vp, _vp], C.c_int),
    "ga_population_steps_f64": ([_vp, _vp, _i64, _i32, _bp, _vp, _vp, _vp], C.c_int),
    "me_first_guess": ([_vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, _vp], C.c_int),
    "me_seeds": ([_vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, _vp, _vp], C.c_int),
    "me_invmax_sigma": ([_vp, _i64, _gp, _i32, C.c_double, _vp, _vp], C.c_int),
    "me_invmax_sigma_f64": ([_vp, _i64, _gp, _i32, C.c_double, _vp, _vp], C.c_int),
    "me_synth_fill": ([_vp, _vp, _i64, _lp, _gp, _i32, _vp, C.POINTER(MeFill), _vp, _vp],
                      C.c_int),
    "me_synth_fill_f64": ([_vp, _vp, _i64, _lp, _gp, _i32, _vp, C.POINTER(MeFill), _vp, _vp],
                          C.c_int),
    "ga_invert_fill": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp, C.POINTER(MeFill), _vp,
                        _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ga_invert_fill_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp, C.POINTER(MeFill),
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "me_prefit_f64": ([_vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, _i32, _vp, _vp, _vp, _vp],
                      C.c_int),
    "me_search_box": ([_vp, _vp, _i64, _lp, _gp, _i32, _bp, _vp, C.c_double, _vp, _vp],
                      C.c_int),
    "mlp_param_count": ([], C.c_int64),
    "mlp_workspace_bytes": ([_i64], C.c_size_t),
    "mlp_init": ([_vp, C.c_uint64, _vp], C.c_int),
    "mlp_features": ([_vp, _i64, _gp, _i32, _vp, _vp], C.c_int),
    "mlp_forward": ([_vp, _vp, _i64, _i32, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "mlp_noalloc_max_rows": ([], _i64),
    "mlp_forward_noalloc": ([_vp, _vp, _i64, _i32, _vp, _vp], C.c_int),
    "mlp_grad": ([_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "mlp_adam": ([_vp, _vp, _vp, _vp, _i32, C.c_float, _vp], C.c_int),
    "mlp_draw_examples": ([C.c_uint64, _i64, _i64, _bp, _vp, _vp, _vp], C.c_int),
    "mlp_add_noise": ([C.c_uint64, _i64, _vp, _i64, _gp, _i32, C.c_float, _vp, _vp], C.c_int),
    "mlp_unscale": ([_vp, _i64, _bp, _vp, _vp], C.c_int),
    "mlp_train_workspace_bytes": ([_i64], C.c_size_t),
    "mlp_train": ([_vp, _vp, _vp, _i32, _i32, _i64, C.c_float, C.c_uint64, _lp, _gp, _i32, _bp,
                   C.c_float, _i32, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "gs_create": ([C.c_size_t, _i32, C.POINTER(_vp)], C.c_int),
    "gs_submit": ([_vp, _vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp, _vp, _vp, _vp,
                   C.POINTER(C.c_uint64)], C.c_int),
    "gs_submit_fill": ([_vp, _vp, _vp, _vp, _i64, _lp, _gp, _i32, _bp, _cp,
                        C.POINTER(MeFill), _vp, _vp, _vp, _vp, C.POINTER(C.c_uint64)], C.c_int),
    "gs_step": ([_vp, _vp], C.c_int),
    "gs_set_max_resident_pixels": ([_vp, _i64], C.c_int),
    "gs_poll": ([_vp, C.c_uint64, C.POINTER(_i32)], C.c_int),
    "gs_cancel": ([_vp, C.c_uint64], C.c_int),
    "gs_release": ([_vp, C.c_uint64], C.c_int),
    "gs_stats": ([_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)],
                 C.c_int),
    "gs_tracked": ([_vp, C.POINTER(C.c_int64)], C.c_int),
    "gs_destroy": ([_vp], C.c_int),
}

EXPORTED = tuple(_SIGS)
ABI_VERSION = 5
STRUCTS = (("me_line", MeLine), ("me_grid", MeGrid), ("me_bounds", MeBounds),
           ("ga_config", GaConfigC), ("me_fill", MeFill))


def lib_path() -> str:
    return _build.SO


def lib():
    """Load libgenesis_hip.so (fails loudly if it has not been built)."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_build.SO):
                raise RuntimeError(
                    "libgenesis_hip.so is not built; run `python -m paper_1208_0302_amd.build` "
                    "(or __graft_entry__.build()) first")
            L = C.CDLL(_build.SO)
            for name, (args, res) in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
            if L.genesis_abi_version() != ABI_VERSION:
                raise RuntimeError(
                    "libgenesis_hip.so has ABI version %d, this binding expects %d; rebuild "
                    "the library from these sources" % (L.genesis_abi_version(), ABI_VERSION))
            # a struct laid out differently here than in the library would
            # hand the device garbage pointers: refuse to run instead
            for which, (sname, struct) in enumerate(STRUCTS):
                if L.genesis_struct_size(which) != C.sizeof(struct):
                    raise RuntimeError(
                        "%s is %d bytes in libgenesis_hip.so but %d in this binding; rebuild "
                        "the library from these sources" % (sname, L.genesis_struct_size(which),
                                                             C.sizeof(struct)))
            _LIB = L
    return _LIB


def _check(rc):
    if rc != ME_OK:
        raise GenesisError(rc, lib().me_last_error().decode())


# --------------------------------------------------------------------------- #
# line data (host only)

def line_from_terms(lambda0_A, Jl, gl, Ju, gu) -> MeLine:
    ln = MeLine()
    _check(lib().me_line_from_terms(float(lambda0_A), float(Jl), float(gl), float(Ju), float(gu),
                                    C.byref(ln)))
    return ln


def line_triplet(lambda0_A, geff) -> MeLine:
    ln = MeLine()
    _check(lib().me_line_triplet(float(lambda0_A), float(geff), C.byref(ln)))
    return ln


def grid(start_A, step_A, n) -> MeGrid:
    return MeGrid(float(start_A), float(step_A), int(n))


def bounds(lo, hi) -> MeBounds:
    b = MeBounds()
    for j in range(NPAR):
        b.lo[j] = float(lo[j])
        b.hi[j] = float(hi[j])
    return b


def _lines(lines: Sequence[MeLine], grids: Sequence[MeGrid]):
    if len(lines) != len(grids):
        raise ValueError("one grid per line")
    la = (MeLine * len(lines))(*lines)
    ga = (MeGrid * len(grids))(*grids)
    return la, ga, len(lines)


def total_samples(grids: Sequence[MeGrid]) -> int:
    return sum(int(g.n) for g in grids)


# --------------------------------------------------------------------------- #
# tensor plumbing

def _stream(t: torch.Tensor):
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: Optional[torch.Tensor], dtype, name, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _real(t: torch.Tensor):
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError("float32 or float64 tensor expected")
    return t.dtype


# --------------------------------------------------------------------------- #
# forward model

def me_synth(params: torch.Tensor, lines, grids, mu=None, out=None, fp16=False, alpha=None,
             fill: Optional[MeFill] = None):
    """Stokes [n, 4, L] from params [n, 9] (Sec. 5 analytic solution).
    fp16=True (float32 tensors only): profiles in packed FP16 (me_synth_f16).
    fill and alpha [n]: the fill-fraction mixture of Sec. 5.2 (me_synth_fill)."""
    dt = _real(params)
    n = params.shape[0]
    L = total_samples(grids)
    _dev(params, dt, "params", (n, NPAR))
    _dev(mu, dt, "mu", (n,))
    if out is None:
        out = torch.empty((n, 4, L), dtype=dt, device=params.device)
    _dev(out, dt, "out", (n, 4, L))
    la, ga, nl = _lines(lines, grids)
    if fill is not None:
        if fp16:
            raise ValueError("the fill fraction needs the native synthesis")
        _dev(alpha, dt, "alpha", (n,))
        f = lib().me_synth_fill if dt == torch.float32 else lib().me_synth_fill_f64
        _check(f(_ptr(params), _ptr(alpha), n, la, ga, nl, _ptr(mu), C.byref(fill), _ptr(out),
                 _stream(params)))
        return out
    if fp16:
        if dt != torch.float32:
            raise ValueError("fp16 synthesis takes float32 parameters")
        f = lib().me_synth_f16
    else:
        f = lib().me_synth if dt == torch.float32 else lib().me_synth_f64
    _check(f(_ptr(params), n, la, ga, nl, _ptr(mu), _ptr(out), _stream(params)))
    return out


def me_chi2(params, obs, sigma, lines, grids, mu=None, out=None):
    """chi-square [npix, pop] of params [npix, pop, 9] (Sec. 5 merit function)."""
    dt = _real(params)
    npix, pop = params.shape[0], params.shape[1]
    L = total_samples(grids)
    _dev(params, dt, "params", (npix, pop, NPAR))
    _dev(obs, dt, "obs", (npix, 4, L))
    _dev(sigma, dt, "sigma", (npix, 4))
    _dev(mu, dt, "mu", (npix,))
    if out is None:
        out = torch.empty((npix, pop), dtype=dt, device=params.device)
    _dev(out, dt, "out", (npix, pop))
    la, ga, nl = _lines(lines, grids)
    f = lib().me_chi2 if dt == torch.float32 else lib().me_chi2_f64
    _check(f(_ptr(params), npix, pop, _ptr(obs), _ptr(sigma), _ptr(mu), la, ga, nl, _ptr(out),
             _stream(params)))
    return out


# --------------------------------------------------------------------------- #
# genetic operators

def ga_init(npix: int, cfg: GAConfig, bnds: Optional[MeBounds] = None, device="cuda"):
    genes = torch.empty((npix, cfg.pop, NPAR), dtype=torch.uint16, device=device)
    c = cfg.c(npix)
    _check(lib().ga_init(npix, C.byref(c), None if bnds is None else C.byref(bnds), _ptr(genes),
                         _stream(genes)))
    return genes


def ga_restart(genes, fitness, cfg: GAConfig, generation: int):
    """Restart of generation `generation` (Sec. 5.6): the worst half replaced by
    Sobol points; returns the new genes (the caller evaluates them)."""
    npix = genes.shape[0]
    dt = _real(fitness)
    _dev(genes, torch.uint16, "genes", (npix, cfg.pop, NPAR))
    _dev(fitness, dt, "fitness", (npix, cfg.pop))
    out = torch.empty_like(genes)
    c = cfg.c(npix)
    f = lib().ga_restart if dt == torch.float32 else lib().ga_restart_f64
    _check(f(_ptr(genes), _ptr(fitness), npix, C.byref(c), int(generation), _ptr(out),
             _stream(genes)))
    return out


def ga_decode(genes: torch.Tensor, bnds: MeBounds):
    _dev(genes, torch.uint16, "genes")
    n = genes.numel() // NPAR
    out = torch.empty(genes.shape, dtype=torch.float32, device=genes.device)
    _check(lib().ga_decode(_ptr(genes), n, C.byref(bnds), _ptr(out), _stream(genes)))
    return out


def ga_evaluate(genes, bnds: MeBounds, obs, sigma, lines, grids, mu=None, out=None):
    dt = _real(obs)
    npix, pop = genes.shape[0], genes.shape[1]
    L = total_samples(grids)
    _dev(genes, torch.uint16, "genes", (npix, pop, NPAR))
    _dev(obs, dt, "obs", (npix, 4, L))
    _dev(sigma, dt, "sigma", (npix, 4))
    _dev(mu, dt, "mu", (npix,))
    if out is None:
        out = torch.empty((npix, pop), dtype=dt, device=genes.device)
    _dev(out, dt, "out", (npix, pop))
    la, ga, nl = _lines(lines, grids)
    f = lib().ga_evaluate if dt == torch.float32 else lib().ga_evaluate_f64
    _check(f(_ptr(genes), npix, pop, C.byref(bnds), _ptr(obs), _ptr(sigma), _ptr(mu), la, ga, nl,
             _ptr(out), _stream(genes)))
    return out


def ga_step(genes_in, fitness, cfg: GAConfig, generation: int, diagnostics=True):
    """One generation of S, R, M with elitism; returns a dict of tensors."""
    dt = _real(fitness)
    npix, pop = genes_in.shape[0], genes_in.shape[1]
    if pop != cfg.pop:
        raise ValueError("genes have pop %d, config says %d" % (pop, cfg.pop))
    _dev(genes_in, torch.uint16, "genes_in", (npix, pop, NPAR))
    _dev(fitness, dt, "fitness", (npix, pop))
    dev = genes_in.device
    out = torch.empty_like(genes_in)
    res = dict(genes=out)
    if diagnostics:
        res.update(parents=torch.empty((npix, pop, 2), dtype=torch.int32, device=dev),
                   xpoint=torch.empty((npix, pop), dtype=torch.int32, device=dev),
                   masks=torch.empty_like(genes_in),
                   elite=torch.empty((npix,), dtype=torch.int32, device=dev))
    c = cfg.c(npix)
    f = lib().ga_step if dt == torch.float32 else lib().ga_step_f64
    _check(f(_ptr(genes_in), _ptr(fitness), npix, C.byref(c), int(generation), _ptr(out),
             _ptr(res.get("parents")), _ptr(res.get("xpoint")), _ptr(res.get("masks")),
             _ptr(res.get("elite")), _stream(genes_in)))
    return res


def ga_workspace_bytes(npix: int, cfg: GAConfig) -> int:
    c = cfg.c(npix)
    return int(lib().ga_workspace_bytes(npix, C.byref(c)))


def ga_invert(obs, sigma, lines, grids, bnds: MeBounds, cfg: GAConfig, mu=None,
              want_population=False, want_status=True, fill: Optional[MeFill] = None):
    """Whole inversion (Algorithm 1) in one launch; returns a dict of tensors.
    fill: the fill fraction of Sec. 5.2 as a tenth fitted parameter
    (ga_invert_fill); the result then has 'alpha' [npix]."""
    dt = _real(obs)
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, dt, "obs", (npix, 4, L))
    _dev(sigma, dt, "sigma", (npix, 4))
    _dev(mu, dt, "mu", (npix,))
    dev = obs.device
    res = dict(params=torch.empty((npix, NPAR), dtype=dt, device=dev),
               chi2=torch.empty((npix,), dtype=dt, device=dev))
    if want_status:
        res["status"] = torch.empty((npix,), dtype=torch.int32, device=dev)
    if want_population:
        res["genes"] = torch.empty((npix, cfg.pop, NPAR), dtype=torch.uint16, device=dev)
        res["fitness"] = torch.empty((npix, cfg.pop), dtype=dt, device=dev)
    la, ga, nl = _lines(lines, grids)
    c = cfg.c(npix)
    if fill is not None:
        res["alpha"] = torch.empty((npix,), dtype=dt, device=dev)
        f = lib().ga_invert_fill if dt == torch.float32 else lib().ga_invert_fill_f64
        _check(f(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl, C.byref(bnds), C.byref(c),
                 C.byref(fill), _ptr(res["params"]), _ptr(res["alpha"]), _ptr(res["chi2"]),
                 _ptr(res.get("status")), _ptr(res.get("genes")), _ptr(res.get("fitness")),
                 _stream(obs)))
        return res
    f = lib().ga_invert if dt == torch.float32 else lib().ga_invert_f64
    _check(f(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl, C.byref(bnds), C.byref(c),
             _ptr(res["params"]), _ptr(res["chi2"]), _ptr(res.get("status")),
             _ptr(res.get("genes")), _ptr(res.get("fitness")), None, 0, _stream(obs)))
    return res


def me_first_guess(obs, lines, grids, bnds: MeBounds, mu=None):
    """Heuristic first guesses [npix, 9] (float32) from float64 observations
    [npix, 4, L] (weak-field, centre-of-gravity and profile-shape estimates,
    Sec. 5.5), for GAConfig.seed_params."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(mu, torch.float64, "mu", (npix,))
    out = torch.empty((npix, NPAR), dtype=torch.float32, device=obs.device)
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_first_guess(_ptr(obs), _ptr(mu), npix, la, ga, nl, C.byref(bnds), _ptr(out),
                                _stream(obs)))
    return out


def me_invmax_sigma(obs, grids, floor=1e-6):
    """Inverse-max weights of Sec. 5.4 as sigma [npix, 4] (the dtype of obs,
    float32 or float64) for observations [npix, 4, L]: the span of I and the
    largest |Q|, |U|, |V| of each pixel, each at least `floor`."""
    npix = obs.shape[0]
    L = total_samples(grids)
    dt = _real(obs)
    _dev(obs, dt, "obs", (npix, 4, L))
    out = torch.empty((npix, 4), dtype=dt, device=obs.device)
    ga = (MeGrid * len(grids))(*grids)
    f = lib().me_invmax_sigma if dt == torch.float32 else lib().me_invmax_sigma_f64
    _check(f(_ptr(obs), npix, ga, len(grids), float(floor), _ptr(out), _stream(obs)))
    return out


SEED_NAMES = ("weak_field", "integral", "centre_of_gravity", "non_magnetic")


def me_seeds(obs, lines, grids, bnds: MeBounds, mu=None, pixel_bounds=None):
    """The four Sec. 5.5 first guesses [npix, 4, 9] (float32; order
    SEED_NAMES, NaN = left random) of observations [npix, 4, L] (float64),
    consistent with pixel_bounds [npix, 2, 9] (float32) when given."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(mu, torch.float64, "mu", (npix,))
    _dev(pixel_bounds, torch.float32, "pixel_bounds", (npix, 2, NPAR))
    out = torch.empty((npix, 4, NPAR), dtype=torch.float32, device=obs.device)
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_seeds(_ptr(obs), _ptr(mu), npix, la, ga, nl, C.byref(bnds),
                          _ptr(pixel_bounds), _ptr(out), _stream(obs)))
    return out


def me_refine_f64(obs, sigma, lines, grids, bnds: MeBounds, params_in, iterations=50, mu=None):
    """FP64 Levenberg-Marquardt refinement of params_in [npix, 9]; returns a
    dict(params, chi2, iters).  obs, sigma, mu and params_in are float64."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(sigma, torch.float64, "sigma", (npix, 4))
    _dev(mu, torch.float64, "mu", (npix,))
    _dev(params_in, torch.float64, "params_in", (npix, NPAR))
    dev = obs.device
    res = dict(params=torch.empty((npix, NPAR), dtype=torch.float64, device=dev),
               chi2=torch.empty((npix,), dtype=torch.float64, device=dev),
               iters=torch.empty((npix,), dtype=torch.int32, device=dev))
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_refine_f64(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl,
                               C.byref(bnds), _ptr(params_in), int(iterations),
                               _ptr(res["params"]), _ptr(res["chi2"]), _ptr(res["iters"]),
                               _stream(obs)))
    return res


def me_refine_fill_f64(obs, sigma, lines, grids, bnds: MeBounds, fill_: MeFill, params_in,
                       alpha_in, iterations=50, mu=None, free_mask=0x3FF):
    """FP64 Levenberg-Marquardt refinement of the fill-fraction model (Sec.
    5.2) over params_in [npix, 9] and alpha_in [npix] (bit 9 of free_mask is
    alpha); returns dict(params, alpha, chi2, iters).  All float64."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(sigma, torch.float64, "sigma", (npix, 4))
    _dev(mu, torch.float64, "mu", (npix,))
    _dev(params_in, torch.float64, "params_in", (npix, NPAR))
    _dev(alpha_in, torch.float64, "alpha_in", (npix,))
    dev = obs.device
    res = dict(params=torch.empty((npix, NPAR), dtype=torch.float64, device=dev),
               alpha=torch.empty((npix,), dtype=torch.float64, device=dev),
               chi2=torch.empty((npix,), dtype=torch.float64, device=dev),
               iters=torch.empty((npix,), dtype=torch.int32, device=dev))
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_refine_fill_f64(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl,
                                    C.byref(bnds), C.byref(fill_), _ptr(params_in),
                                    _ptr(alpha_in), int(iterations), int(free_mask),
                                    _ptr(res["params"]), _ptr(res["alpha"]), _ptr(res["chi2"]),
                                    _ptr(res["iters"]), _stream(obs)))
    return res


def me_uncertainty_f64(obs, sigma, lines, grids, bnds: MeBounds, params_opt, steps, mu=None,
                       free_mask=0x1FF, want_hessian=False):
    """Sec. 6 uncertainties [npix, 9] at params_opt [npix, 9] from initial
    steps [npix, 9] (e.g. ga_population_steps); returns dict(sigma, steps[,
    hessian, hessian_err]).  All float64."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(sigma, torch.float64, "sigma", (npix, 4))
    _dev(mu, torch.float64, "mu", (npix,))
    _dev(params_opt, torch.float64, "params_opt", (npix, NPAR))
    _dev(steps, torch.float64, "steps", (npix, NPAR))
    dev = obs.device
    res = dict(sigma=torch.empty((npix, NPAR), dtype=torch.float64, device=dev),
               steps=torch.empty((npix, NPAR), dtype=torch.float64, device=dev))
    if want_hessian:
        res["hessian"] = torch.empty((npix, NPAR, NPAR), dtype=torch.float64, device=dev)
        res["hessian_err"] = torch.empty((npix, NPAR, NPAR), dtype=torch.float64, device=dev)
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_uncertainty_f64(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl,
                                    C.byref(bnds), _ptr(params_opt), _ptr(steps),
                                    int(free_mask), _ptr(res["sigma"]), _ptr(res.get("hessian")),
                                    _ptr(res.get("hessian_err")), _ptr(res["steps"]),
                                    _stream(obs)))
    return res


def ga_population_steps(genes, fitness, bnds: MeBounds, params_opt):
    """Sec. 6 initial steps [npix, 9] (float64) from a final population:
    genes [npix, pop, 9] uint16, fitness [npix, pop] float32 or float64,
    params_opt [npix, 9] float64."""
    npix, pop = genes.shape[0], genes.shape[1]
    _dev(genes, torch.uint16, "genes", (npix, pop, NPAR))
    _dev(params_opt, torch.float64, "params_opt", (npix, NPAR))
    if fitness.dtype not in (torch.float32, torch.float64):
        raise TypeError("fitness must be float32 or float64")
    _dev(fitness, fitness.dtype, "fitness", (npix, pop))
    out = torch.empty((npix, NPAR), dtype=torch.float64, device=genes.device)
    f = {torch.float32: lib().ga_population_steps,
         torch.float64: lib().ga_population_steps_f64}[fitness.dtype]
    _check(f(_ptr(genes), _ptr(fitness), npix, pop, C.byref(bnds), _ptr(params_opt), _ptr(out),
             _stream(genes)))
    return out


def me_prefit_f64(obs, sigma, lines, grids, bnds: MeBounds, params_in, iterations=30, mu=None):
    """Non-magnetic pre-fit (Sec. 5.3): Levenberg-Marquardt with B held at 0,
    adjusting v_los, Doppler width, damping, eta0, S0 and S1 from params_in
    [npix, 9] (float64); returns dict(params, chi2, iters)."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(sigma, torch.float64, "sigma", (npix, 4))
    _dev(mu, torch.float64, "mu", (npix,))
    _dev(params_in, torch.float64, "params_in", (npix, NPAR))
    dev = obs.device
    res = dict(params=torch.empty((npix, NPAR), dtype=torch.float64, device=dev),
               chi2=torch.empty((npix,), dtype=torch.float64, device=dev),
               iters=torch.empty((npix,), dtype=torch.int32, device=dev))
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_prefit_f64(_ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl,
                               C.byref(bnds), _ptr(params_in), int(iterations),
                               _ptr(res["params"]), _ptr(res["chi2"]), _ptr(res["iters"]),
                               _stream(obs)))
    return res


def me_search_box(obs, sigma, lines, grids, bnds: MeBounds, prefit=None, polarity_nsigma=3.0):
    """Per-pixel search boxes [npix, 2, 9] (float32) for GAConfig.pixel_bounds:
    pre-fit ranges (Sec. 5.3) from prefit [npix, 9] (float64, may be None) and
    the polarity restriction (Sec. 5.5) where Stokes V's first moment exceeds
    polarity_nsigma noise deviations (<= 0: none)."""
    npix = obs.shape[0]
    L = total_samples(grids)
    _dev(obs, torch.float64, "obs", (npix, 4, L))
    _dev(sigma, torch.float64, "sigma", (npix, 4))
    _dev(prefit, torch.float64, "prefit", (npix, NPAR))
    out = torch.empty((npix, 2, NPAR), dtype=torch.float32, device=obs.device)
    la, ga, nl = _lines(lines, grids)
    _check(lib().me_search_box(_ptr(obs), _ptr(sigma), npix, la, ga, nl, C.byref(bnds),
                               _ptr(prefit), float(polarity_nsigma), _ptr(out), _stream(obs)))
    return out


class ServingSession:
    """Continuous-batching inversion service (gs_* in the C ABI).

    submit() queues a tile and returns its id; step() admits what fits in the
    memory budget and advances every resident tile by `gens_per_step`
    generations; poll() tells when a tile's outputs are ready; result()
    returns them and releases the request (the session then holds no
    reference to its tensors); release() forgets a cancelled request.  The
    input tensors of a request are kept alive here until then, because the
    device reads them until the request finishes."""

    def __init__(self, budget_bytes: int, gens_per_step: int = 10, device="cuda",
                 max_resident_pixels: int = 0):
        self._h = _vp()
        self.device = torch.device(device)
        _check(lib().gs_create(int(budget_bytes), int(gens_per_step), C.byref(self._h)))
        self._req = {}
        if max_resident_pixels:
            _check(lib().gs_set_max_resident_pixels(self._h, int(max_resident_pixels)))

    def submit(self, obs, sigma, lines, grids, bnds: MeBounds, cfg: GAConfig, mu=None,
               fill: MeFill = None):
        """Queue a tile; cfg.synth_precision chooses FP16 profile synthesis,
        `fill` the fill-fraction merit of Sec. 5.2 (the result then has
        'alpha')."""
        npix = obs.shape[0]
        L = total_samples(grids)
        _dev(obs, torch.float32, "obs", (npix, 4, L))
        _dev(sigma, torch.float32, "sigma", (npix, 4))
        _dev(mu, torch.float32, "mu", (npix,))
        out = dict(params=torch.empty((npix, NPAR), dtype=torch.float32, device=obs.device),
                   chi2=torch.empty((npix,), dtype=torch.float32, device=obs.device),
                   status=torch.empty((npix,), dtype=torch.int32, device=obs.device))
        la, ga, nl = _lines(lines, grids)
        c = cfg.c(npix)
        rid = C.c_uint64()
        if fill is None:
            _check(lib().gs_submit(self._h, _ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga, nl,
                                   C.byref(bnds), C.byref(c), _ptr(out["params"]),
                                   _ptr(out["chi2"]), _ptr(out["status"]), C.byref(rid)))
        else:
            out["alpha"] = torch.empty((npix,), dtype=torch.float32, device=obs.device)
            _check(lib().gs_submit_fill(self._h, _ptr(obs), _ptr(sigma), _ptr(mu), npix, la, ga,
                                        nl, C.byref(bnds), C.byref(c), C.byref(fill),
                                        _ptr(out["params"]), _ptr(out["alpha"]),
                                        _ptr(out["chi2"]), _ptr(out["status"]), C.byref(rid)))
        # the device reads the inputs and writes the outputs until the request
        # is done: keep them alive until it is released
        self._req[rid.value] = dict(out=out, keep=(obs, sigma, mu, cfg.seed_params,
                                                    cfg.pixel_bounds))
        return rid.value

    def step(self):
        _check(lib().gs_step(self._h, _vp(torch.cuda.current_stream(self.device).cuda_stream)))

    def poll(self, rid) -> int:
        d = _i32()
        _check(lib().gs_poll(self._h, C.c_uint64(rid), C.byref(d)))
        return int(d.value)

    def cancel(self, rid):
        _check(lib().gs_cancel(self._h, C.c_uint64(rid)))

    def stats(self):
        q, r, b = C.c_int64(), C.c_int64(), C.c_size_t()
        _check(lib().gs_stats(self._h, C.byref(q), C.byref(r), C.byref(b)))
        return dict(queued=q.value, resident=r.value, bytes_in_use=b.value)

    def tracked(self) -> int:
        """Requests the library still holds records of."""
        n = C.c_int64()
        _check(lib().gs_tracked(self._h, C.byref(n)))
        return int(n.value)

    def held(self) -> int:
        """Requests whose tensors this object still keeps alive."""
        return len(self._req)

    def release(self, rid):
        """Forget a finished (poll() == 1) or cancelled (-1) request and drop
        the references to its tensors."""
        _check(lib().gs_release(self._h, C.c_uint64(rid)))
        self._req.pop(rid, None)

    def result(self, rid):
        """Outputs of a finished request (poll() must have given 1); the
        request is released."""
        if self.poll(rid) != 1:
            raise GenesisError(ME_EBUSY, "request %d is not finished" % rid)
        out = self._req[rid]["out"]
        self.release(rid)
        return out

    def close(self):
        if self._h:
            lib().gs_destroy(self._h)
            self._h = _vp()
            self._req.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The learned proposal network (mlp_* in the C ABI): FP32 master weights,
    Adam moments and a workspace on the device; every step runs in the
    library's kernels (MFMA BF16 products by default, precision=1 for FP32)."""

    def __init__(self, seed=0, device="cuda", precision=0):
        self.device = torch.device(device)
        self.precision = precision
        self.n = int(lib().mlp_param_count())
        self.master = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step_no = 0
        self._ws = None
        self._ws_batch = 0
        _check(lib().mlp_init(_ptr(self.master), int(seed), _stream(self.master)))

    def _workspace(self, batch):
        if self._ws is None or self._ws_batch < batch:
            nb = int(lib().mlp_workspace_bytes(int(batch)))
            self._ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            self._ws_batch = batch
        return self._ws, int(lib().mlp_workspace_bytes(int(self._ws_batch)))

    def features(self, obs, grids):
        npix = obs.shape[0]
        _dev(obs, torch.float32, "obs")
        x = torch.empty((npix, 1024), dtype=torch.float32, device=obs.device)
        ga = (MeGrid * len(grids))(*grids)
        _check(lib().mlp_features(_ptr(obs), npix, ga, len(grids), _ptr(x), _stream(obs)))
        return x

    def forward(self, x, precision=None):
        n = x.shape[0]
        _dev(x, torch.float32, "x", (n, 1024))
        y = torch.empty((n, NPAR), dtype=torch.float32, device=x.device)
        ws, nb = self._workspace(n)
        _check(lib().mlp_forward(_ptr(self.master), _ptr(x), n,
                                 self.precision if precision is None else precision, _ptr(y),
                                 _ptr(ws), nb, _stream(x)))
        return y

    def forward_noalloc(self, x, precision=None):
        """forward() through mlp_forward_noalloc: the library's own device
        scratch instead of a workspace (at most mlp_noalloc_max_rows() rows)."""
        n = x.shape[0]
        _dev(x, torch.float32, "x", (n, 1024))
        y = torch.empty((n, NPAR), dtype=torch.float32, device=x.device)
        _check(lib().mlp_forward_noalloc(_ptr(self.master), _ptr(x), n,
                                         self.precision if precision is None else precision,
                                         _ptr(y), _stream(x)))
        return y

    def compute_grad(self, x, target, precision=None):
        b = x.shape[0]
        _dev(x, torch.float32, "x", (b, 1024))
        _dev(target, torch.float32, "target", (b, NPAR))
        ws, nb = self._workspace(b)
        _check(lib().mlp_grad(_ptr(self.master), _ptr(x), _ptr(target), b,
                              self.precision if precision is None else precision,
                              _ptr(self.grad), _ptr(self.loss), _ptr(ws), nb, _stream(x)))
        return self.grad, self.loss

    def adam(self, lr):
        self.step_no += 1
        _check(lib().mlp_adam(_ptr(self.master), _ptr(self.m), _ptr(self.v), _ptr(self.grad),
                              self.step_no, float(lr), _stream(self.master)))

    def examples(self, seed, first, n, lines, grids, bnds, sigma_rel=1e-3):
        """n noisy synthetic training pairs (features, scaled targets), drawn,
        synthesised and normalised on the device."""
        params = torch.empty((n, NPAR), dtype=torch.float32, device=self.device)
        target = torch.empty_like(params)
        _check(lib().mlp_draw_examples(int(seed), int(first), n, C.byref(bnds), _ptr(params),
                                       _ptr(target), _stream(params)))
        stokes = me_synth(params, lines, grids)
        ga = (MeGrid * len(grids))(*grids)
        _check(lib().mlp_add_noise(int(seed), int(first), _ptr(params), n, ga, len(grids),
                                   float(sigma_rel), _ptr(stokes), _stream(params)))
        return self.features(stokes, grids), target

    def train(self, lines, grids, bnds, steps, batch=512, lr=1e-3, seed=1, sigma_rel=1e-3):
        """`steps` Adam steps on fresh synthetic examples (one library call);
        returns the per-step losses as a device tensor."""
        nb = int(lib().mlp_train_workspace_bytes(int(batch)))
        if getattr(self, "_tws", None) is None or self._tws.numel() < nb:
            self._tws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        losses = torch.empty(max(int(steps), 1), dtype=torch.float32, device=self.device)
        la, ga, nl = _lines(lines, grids)
        _check(lib().mlp_train(_ptr(self.master), _ptr(self.m), _ptr(self.v), self.step_no + 1,
                               int(steps), int(batch), float(lr), int(seed), la, ga, nl,
                               C.byref(bnds), float(sigma_rel), self.precision, _ptr(losses),
                               _ptr(self._tws), self._tws.numel(), _stream(self.master)))
        self.step_no += int(steps)
        return losses[:steps]

    def predict(self, obs, grids, bnds):
        """First-guess parameters [npix, 9] for observations [npix, 4, L]."""
        y = self.forward(self.features(obs, grids))
        params = torch.empty_like(y)
        _check(lib().mlp_unscale(_ptr(y), y.shape[0], C.byref(bnds), _ptr(params), _stream(y)))
        return params
