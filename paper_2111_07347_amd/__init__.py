"""MI355X-native template-matching orientation mapping (Pyxem method,
arXiv 2111.07347), Python binding of libtm.

Argument marshalling only: every step runs in libtm's HIP kernels. PyTorch
provides device memory and the current HIP stream. Names follow the C ABI in
include/tm.h:

    grid = PolarGrid(R=128, n_theta=360, cx=128.0, cy=128.0)
    lib = Library(kx, ky, intensity, offsets, px_per_inv_angstrom, grid)
    polar, norms, prof = polar_transform(patterns, grid)
    top_t, top_s, top_q = match_batch(lib, polar, norms, N=5)
    top_t, top_s, top_q = topn(best_score, best_angle, N=5)

The library must have been built (``python paper_2111_07347_amd/build.py``);
importing without it raises ImportError. There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

TM_OK, TM_EINVAL, TM_ENOMEM, TM_EHIP, TM_ENODEV, TM_EUNSUPPORTED, TM_ENOMEM_BUDGET = (
    0, -1, -2, -3, -4, -5, -6)
TM_U16, TM_F32 = 0, 1
TM_PREC_FP32, TM_PREC_BF16, TM_PREC_FP16, TM_PREC_FP8 = 0, 1, 2, 3
TM_LIB_MIRROR, TM_LIB_UNIT_INTENSITY, TM_LIB_KEEP_DIRECT_BEAM, TM_LIB_NO_GROUPING = 1, 2, 4, 8
TM_LIB_FFT = 16
TM_COARSE_NONE, TM_COARSE_FFT, TM_COARSE_BOUND = 0, 1, 2
TM_RESCORE_CERTIFIED, TM_RESCORE_KEEP = 0, 1
TM_MAX_N = 64
TM_LAUE_M3M, TM_LAUE_MMM, TM_LAUE_6MMM = 0, 1, 2
LAUE_GROUPS = {"m-3m": TM_LAUE_M3M, "mmm": TM_LAUE_MMM, "6/mmm": TM_LAUE_6MMM}

EXPORTED = ("tm_load_library", "tm_free_library", "tm_library_info", "tm_library_layout",
            "tm_library_rows", "tm_polar_transform", "tm_polar_transform_rows",
            "tm_mask_from_mean", "tm_match_batch", "tm_match_batch_static", "tm_refine_angles", "tm_prefilter", "tm_match_candidates",
            "tm_fft_scores", "tm_fft_error_bound", "tm_bound_scores", "tm_bound_scores_slots", "tm_bound_layout", "tm_orientations", "tm_ipf_deviation",
            "tm_simulate_library", "tm_preprocess",
            "tm_topn", "tm_last_error", "tm_version")


class TMError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("r0", ctypes.c_double),
                ("dr", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("interp", ctypes.c_int32)]


class _PreOpts(ctypes.Structure):
    _fields_ = [("r_box", ctypes.c_int32), ("frac", ctypes.c_double),
                ("sigma_min", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("sigma_blur", ctypes.c_double), ("threshold", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("prefilter_keep", ctypes.c_double), ("prefilter_prec", ctypes.c_int32),
                ("coarse", ctypes.c_int32), ("rescore_policy", ctypes.c_int32),
                ("compact_rows", ctypes.c_int32), ("rescore_keep", ctypes.c_double),
                ("n_rescored", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2111_07347_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, F = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                         ctypes.c_float)
    sig = {
        "tm_load_library": [P, P, P, P, I32, D, ctypes.POINTER(_Grid), ctypes.c_uint32, P,
                            ctypes.POINTER(P)],
        "tm_free_library": [P],
        "tm_library_info": [P, P, P, P],
        "tm_library_layout": [P, P, P, P, P, P],
        "tm_library_rows": [P, P, ctypes.POINTER(P)],
        "tm_polar_transform": [P, ctypes.c_int, I32, I32, I32, ctypes.POINTER(_Grid), F, F, P, P,
                               P, P],
        "tm_polar_transform_rows": [P, ctypes.c_int, I32, I32, I32, ctypes.POINTER(_Grid), F, F,
                                    P, P, I32, P, P, P, P],
        "tm_mask_from_mean": [P, ctypes.c_int, I32, I32, I32, D, I32, I32, P, P],
        "tm_match_batch": [P, P, P, P, I32, ctypes.POINTER(_Opts), I32, P, P, P, P, P, P],
        "tm_match_batch_static": [P, P, P, P, I32, ctypes.POINTER(_Opts), I32, P, P, P, P, P, P],
        "tm_bound_scores": [P, P, P, I32, I32, P, P],
        "tm_bound_layout": [P, P, P, P],
        "tm_bound_scores_slots": [P, P, P, I32, I32, P, P, P],
        "tm_prefilter": [P, P, I32, I32, I32, P, P],
        "tm_match_candidates": [P, P, P, I32, P, I32, I32, P, P, P, P],
        "tm_fft_scores": [P, P, P, I32, I32, P, P, P],
        "tm_refine_angles": [P, P, P, I32, I32, I32, P, P, P, P],
        "tm_fft_error_bound": [P, ctypes.POINTER(D)],
        "tm_orientations": [P, I32, I32, I32, P, P, P, I32, I32, P, P],
        "tm_ipf_deviation": [P, I32, P, I32, I32, I32, P, P],
        "tm_simulate_library": [P, P, P, I32, D, P, I32, D, D, D, D, I32, P, P, P, P, P],
        "tm_preprocess": [P, ctypes.c_int, I32, I32, I32, ctypes.POINTER(_PreOpts), P, P, P],
        "tm_topn": [P, P, I32, I32, I32, P, P, P, P],
        "tm_last_error": [],
        "tm_version": [],
    }
    for name, args in sig.items():
        if not hasattr(lib, name):
            raise ImportError(f"{LIB_PATH} lacks {name}: it is stale, rebuild it with "
                              "`python paper_2111_07347_amd/build.py`")
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("tm_last_error", "tm_version") else ctypes.c_int
    return lib


_lib = _load()


def version() -> str:
    return _lib.tm_version().decode()


def last_error() -> str:
    return _lib.tm_last_error().decode()


def _check(code: int, where: str):
    if code != TM_OK:
        raise TMError(code, where, last_error())


@dataclass(frozen=True)
class PolarGrid:
    """Polar sampling grid: r_j = r0 + j*dr, theta_k = 2 pi k / n_theta, about
    (cx, cy) in pixel-index coordinates (x = column, y = row)."""
    R: int
    n_theta: int = 360
    cx: float = 0.0
    cy: float = 0.0
    r0: float = 0.0
    dr: float = 1.0
    interp: str = "bilinear"

    def _c(self) -> _Grid:
        if self.interp not in ("bilinear", "nearest"):
            raise ValueError(f"interp must be 'bilinear' or 'nearest', not {self.interp!r}")
        return _Grid(int(self.R), int(self.n_theta), float(self.r0), float(self.dr),
                     float(self.cx), float(self.cy), 1 if self.interp == "bilinear" else 0)


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _require(t, name, dtype, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Library:
    """Device-resident template library (tm_load_library).

    kx, ky, intensity: spot coordinates (1/Angstrom) and intensities of all
    templates concatenated; offsets: CSR offsets [T+1]."""

    def __init__(self, kx, ky, intensity, offsets, px_per_inv_angstrom: float, grid: PolarGrid,
                 mirror: bool = True, unit_intensity: bool = False,
                 keep_direct_beam: bool = False, grouping: bool = True, fft: bool = False,
                 stream=None):
        kx = np.ascontiguousarray(kx, dtype=np.float64)
        ky = np.ascontiguousarray(ky, dtype=np.float64)
        inten = np.ascontiguousarray(intensity, dtype=np.float64)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if not (len(kx) == len(ky) == len(inten) == int(off[-1])):
            raise ValueError("kx, ky, intensity must all have offsets[-1] entries")
        flags = ((TM_LIB_MIRROR if mirror else 0) | (TM_LIB_UNIT_INTENSITY if unit_intensity else 0)
                 | (TM_LIB_KEEP_DIRECT_BEAM if keep_direct_beam else 0)
                 | (0 if grouping else TM_LIB_NO_GROUPING) | (TM_LIB_FFT if fft else 0))
        self.grid = grid
        self.T = len(off) - 1
        self.mirror = mirror
        h = ctypes.c_void_p()
        g = grid._c()
        _check(_lib.tm_load_library(kx.ctypes.data, ky.ctypes.data, inten.ctypes.data,
                                    off.ctypes.data, self.T, float(px_per_inv_angstrom),
                                    ctypes.byref(g), flags, _stream_ptr(stream), ctypes.byref(h)),
               "tm_load_library")
        self._h = h

    @property
    def handle(self) -> int:
        return self._h.value

    def info(self):
        tt, ns, db = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
        _check(_lib.tm_library_info(self._h, ctypes.byref(tt), ctypes.byref(ns), ctypes.byref(db)),
               "tm_library_info")
        return {"n_templates_total": tt.value, "n_spots": ns.value, "device_bytes": db.value}

    def layout(self):
        g, nb, nr, rw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rec = ctypes.c_int64()
        _check(_lib.tm_library_layout(self._h, ctypes.byref(g), ctypes.byref(nb), ctypes.byref(nr),
                                      ctypes.byref(rec), ctypes.byref(rw)), "tm_library_layout")
        n_theta = self.grid.n_theta
        return {"group": g.value, "n_bands": nb.value, "n_rows": nr.value, "n_records": rec.value,
                "row_width": rw.value, "narrow": rw.value == n_theta + 63}

    def bound_layout(self):
        """tm_bound_layout: the window-bound data's chunks, record units per
        pattern and coarse window width (TMError if the library has none)."""
        ch, un, w = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.tm_bound_layout(self._h, ctypes.byref(ch), ctypes.byref(un), ctypes.byref(w)),
               "tm_bound_layout")
        return {"chunks": ch.value, "units": un.value, "win": w.value}

    def rows(self):
        """tm_library_rows: (number of polar rows the templates touch, device
        address of the library's [R] int32 row map)."""
        if getattr(self, "_rows", None) is None:
            n, m = ctypes.c_int32(), ctypes.c_void_p()
            _check(_lib.tm_library_rows(self._h, ctypes.byref(n), ctypes.byref(m)), "tm_library_rows")
            self._rows = (n.value, m.value)
        return self._rows

    def fft_error_bound(self) -> float:
        """tm_fft_error_bound: certified bound on |Q~ - Q32| of the Fourier
        route (library loaded with fft=True)."""
        e = ctypes.c_double()
        _check(_lib.tm_fft_error_bound(self._h, ctypes.byref(e)), "tm_fft_error_bound")
        return e.value

    @property
    def n_total(self) -> int:
        return self.info()["n_templates_total"]

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tm_free_library(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def polar_transform(patterns, grid: PolarGrid, gamma: float = 1.0, subtract: float = 0.0,
                    polar_out=None, norm_out=None, profile_out=None, want_profile: bool = True,
                    lib: "Library | None" = None, mask=None, stream=None):
    """tm_polar_transform on a [B, H, W] uint16/float32 device tensor.
    Returns (polar [B, R, n_theta] f32, norms [B] f64, profiles [R, B] f32 or None).
    With lib (tm_polar_transform_rows), polar holds only the rows lib's
    templates touch: [B, n_rows, n_theta]; norms and profiles still cover
    all R rows. mask, an [H, W] float32 device tensor, multiplies every
    transformed pattern before resampling (two-stage indexing)."""
    torch = _torch()
    if patterns.dtype == torch.float32:
        dt = TM_F32
    elif patterns.dtype in (torch.uint16, torch.int16):
        dt = TM_U16
    else:
        raise TypeError("patterns must be float32 or uint16")
    if patterns.dim() != 3:
        raise ValueError("patterns must be [B, H, W]")
    if not patterns.is_cuda or not patterns.is_contiguous():
        raise ValueError("patterns must be a contiguous device tensor")
    B, H, W = patterns.shape
    dev = patterns.device
    n_out, row_map = grid.R, None
    if lib is not None and lib.rows()[0] > 0:
        n_out, row_map = lib.rows()
    if polar_out is None:
        polar_out = torch.empty((B, n_out, grid.n_theta), dtype=torch.float32, device=dev)
    if norm_out is None:
        norm_out = torch.empty((B,), dtype=torch.float64, device=dev)
    if profile_out is None and want_profile:
        profile_out = torch.empty((grid.R, B), dtype=torch.float32, device=dev)
    _require(polar_out, "polar_out", torch.float32, (B, n_out, grid.n_theta))
    _require(norm_out, "norm_out", torch.float64, (B,))
    if profile_out is not None:
        _require(profile_out, "profile_out", torch.float32, (grid.R, B))
    g = grid._c()
    if mask is not None:
        _require(mask, "mask", torch.float32, (H, W))
    if row_map is None and mask is None:
        _check(_lib.tm_polar_transform(_ptr(patterns), dt, B, H, W, ctypes.byref(g), float(gamma),
                                       float(subtract), _ptr(polar_out), _ptr(norm_out),
                                       _ptr(profile_out), _stream_ptr(stream)), "tm_polar_transform")
    else:
        _check(_lib.tm_polar_transform_rows(_ptr(patterns), dt, B, H, W, ctypes.byref(g),
                                            float(gamma), float(subtract), _ptr(mask), row_map,
                                            int(n_out), _ptr(polar_out), _ptr(norm_out),
                                            _ptr(profile_out), _stream_ptr(stream)),
               "tm_polar_transform_rows")
    return polar_out, norm_out, profile_out


def mask_from_mean(patterns, threshold: float, n_open: int = 1, n_grow: int = 2, stream=None):
    """tm_mask_from_mean: [H, W] float32 mask (1 keep, 0 masked) of the
    pixels that are bright in the average of the [B, H, W] patterns, after an
    opening and n_grow dilations."""
    torch = _torch()
    if patterns.dtype == torch.float32:
        dt = TM_F32
    elif patterns.dtype in (torch.uint16, torch.int16):
        dt = TM_U16
    else:
        raise TypeError("patterns must be float32 or uint16")
    _require(patterns, "patterns", patterns.dtype)
    B, H, W = patterns.shape
    out = torch.empty((H, W), dtype=torch.float32, device=patterns.device)
    _check(_lib.tm_mask_from_mean(_ptr(patterns), dt, B, H, W, float(threshold), int(n_open),
                                  int(n_grow), _ptr(out), _stream_ptr(stream)),
           "tm_mask_from_mean")
    return out


def _layout(lib: "Library", polar) -> int:
    """1 if polar holds only lib's touched rows, 0 if all R rows."""
    rows = polar.shape[1]
    if rows == lib.grid.R:
        return 0
    if rows == lib.rows()[0]:
        return 1
    raise ValueError(f"polar has {rows} rows: expected R={lib.grid.R} or the library's "
                     f"{lib.rows()[0]} touched rows")


COARSE = {None: TM_COARSE_NONE, "none": TM_COARSE_NONE, "fft": TM_COARSE_FFT,
          "bound": TM_COARSE_BOUND}
RESCORE = {"certified": TM_RESCORE_CERTIFIED, "keep": TM_RESCORE_KEEP}


def _opts(prefilter_keep: float, prefilter_prec: int, coarse: int = TM_COARSE_NONE,
          rescore: int = TM_RESCORE_CERTIFIED, rescore_keep: float = 0.0, n_rescored=None,
          compact: int = 0):
    if prefilter_keep == 0.0 and coarse == TM_COARSE_NONE and n_rescored is None and not compact:
        return None
    o = _Opts()
    o.compact_rows = int(compact)
    o.prefilter_keep = float(prefilter_keep)
    o.prefilter_prec = int(prefilter_prec)
    o.coarse = int(coarse)
    o.rescore_policy = int(rescore)
    o.rescore_keep = float(rescore_keep)
    o.n_rescored = _ptr(n_rescored) or None
    return o


def match_batch(lib: Library, polar, norms, N: int, profiles=None, prefilter_keep: float = 0.0,
                prefilter_prec: int = TM_PREC_FP32, with_best: bool = False, out=None,
                coarse=None, rescore="certified", rescore_keep: float = 0.0,
                n_rescored=None, stream=None):
    """tm_match_batch. Returns (top_template [B,N] i32, top_angle [B,N] i32,
    top_score [B,N] f32) and, with with_best, also (best_score [B,T'] f32,
    best_angle [B,T'] i16). coarse="fft" scores every template through the
    Fourier route first and rescores candidates exactly (rescore="certified"
    or "keep" with rescore_keep); n_rescored, a [B] int32 device tensor, if
    given receives the number of templates scored exactly per pattern."""
    torch = _torch()
    B = polar.shape[0]
    compact = _layout(lib, polar)
    _require(polar, "polar", torch.float32, (B, polar.shape[1], lib.grid.n_theta))
    _require(norms, "norms", torch.float64, (B,))
    if profiles is not None:
        _require(profiles, "profiles", torch.float32, (lib.grid.R, B))
    dev = polar.device
    if out is None:
        out = (torch.empty((B, N), dtype=torch.int32, device=dev),
               torch.empty((B, N), dtype=torch.int32, device=dev),
               torch.empty((B, N), dtype=torch.float32, device=dev))
    tt, ts, tq = out
    _require(tt, "top_template", torch.int32, (B, N))
    _require(ts, "top_angle", torch.int32, (B, N))
    _require(tq, "top_score", torch.float32, (B, N))
    bq = bs = None
    if with_best:
        Tn = lib.n_total
        bq = torch.empty((B, Tn), dtype=torch.float32, device=dev)
        bs = torch.empty((B, Tn), dtype=torch.int16, device=dev)
    if n_rescored is not None:
        _require(n_rescored, "n_rescored", torch.int32, (B,))
    o = _opts(prefilter_keep, _prec(prefilter_prec), COARSE[coarse],
              RESCORE[rescore] if isinstance(rescore, str) else int(rescore), rescore_keep,
              n_rescored, compact)
    _check(_lib.tm_match_batch(lib._h, _ptr(polar), _ptr(norms), _ptr(profiles), B,
                               ctypes.byref(o) if o is not None else None, int(N), _ptr(tt),
                               _ptr(ts), _ptr(tq), _ptr(bq), _ptr(bs), _stream_ptr(stream)),
           "tm_match_batch")
    return (tt, ts, tq, bq, bs) if with_best else (tt, ts, tq)


PRECISIONS = {"fp32": TM_PREC_FP32, "bf16": TM_PREC_BF16, "fp16": TM_PREC_FP16, "fp8": TM_PREC_FP8}


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def prefilter(lib: Library, profiles, n_keep: int, precision="fp32", stream=None):
    """tm_prefilter: per pattern the n_keep base templates whose radial
    profile correlates best with the pattern's. Returns [B, n_keep] int32
    (ascending template indices)."""
    torch = _torch()
    R, B = profiles.shape
    _require(profiles, "profiles", torch.float32, (lib.grid.R, B))
    kept = torch.empty((B, n_keep), dtype=torch.int32, device=profiles.device)
    _check(_lib.tm_prefilter(lib._h, _ptr(profiles), B, int(n_keep), _prec(precision), _ptr(kept),
                             _stream_ptr(stream)), "tm_prefilter")
    return kept


def match_candidates(lib: Library, polar, norms, candidates, N: int, stream=None):
    """tm_match_candidates: exact search over per-pattern candidate template
    lists [B, n_cand] (int32). Returns (template, angle, score) [B, N]."""
    torch = _torch()
    B = polar.shape[0]
    _require(polar, "polar", torch.float32, (B, lib.grid.R, lib.grid.n_theta))
    _require(norms, "norms", torch.float64, (B,))
    _require(candidates, "candidates", torch.int32)
    if candidates.shape[0] != B:
        raise ValueError("candidates must have one row per pattern")
    dev = polar.device
    tt = torch.empty((B, N), dtype=torch.int32, device=dev)
    ts = torch.empty((B, N), dtype=torch.int32, device=dev)
    tq = torch.empty((B, N), dtype=torch.float32, device=dev)
    _check(_lib.tm_match_candidates(lib._h, _ptr(polar), _ptr(norms), B, _ptr(candidates),
                                    candidates.shape[1], int(N), _ptr(tt), _ptr(ts), _ptr(tq),
                                    _stream_ptr(stream)), "tm_match_candidates")
    return tt, ts, tq


def refine_angles(lib: Library, polar, norms, top_template, top_angle, stream=None):
    """tm_refine_angles: sub-bin in-plane angles (degrees, [B, N] float32) of
    the matches (top_template, top_angle) from match_batch."""
    torch = _torch()
    B = polar.shape[0]
    compact = _layout(lib, polar)
    _require(norms, "norms", torch.float64, (B,))
    _require(top_template, "top_template", torch.int32)
    N = top_template.shape[1]
    _require(top_template, "top_template", torch.int32, (B, N))
    _require(top_angle, "top_angle", torch.int32, (B, N))
    out = torch.empty((B, N), dtype=torch.float32, device=polar.device)
    _check(_lib.tm_refine_angles(lib._h, _ptr(polar), _ptr(norms), B, compact, int(N),
                                 _ptr(top_template), _ptr(top_angle), _ptr(out),
                                 _stream_ptr(stream)), "tm_refine_angles")
    return out


def orientations(lib_euler, top_template, top_angle=None, angle_deg=None, n_theta: int = 360,
                 mirrors: bool = True, stream=None):
    """tm_orientations: Bunge angles (phi1, Phi, phi2) in radians, [B, N, 3]
    float64, of matches (top_template with either angle bins top_angle or
    refined angles angle_deg in degrees). lib_euler: [T, 2] float64 device
    tensor of the base templates' (Phi, phi2)."""
    torch = _torch()
    _require(lib_euler, "lib_euler", torch.float64)
    T = lib_euler.shape[0]
    _require(lib_euler, "lib_euler", torch.float64, (T, 2))
    _require(top_template, "top_template", torch.int32)
    B, N = top_template.shape
    if (top_angle is None) == (angle_deg is None):
        raise ValueError("give exactly one of top_angle and angle_deg")
    if top_angle is not None:
        _require(top_angle, "top_angle", torch.int32, (B, N))
    else:
        _require(angle_deg, "angle_deg", torch.float32, (B, N))
    out = torch.empty((B, N, 3), dtype=torch.float64, device=top_template.device)
    _check(_lib.tm_orientations(_ptr(lib_euler), int(T), 1 if mirrors else 0, int(n_theta),
                                _ptr(top_template), _ptr(top_angle), _ptr(angle_deg), int(B),
                                int(N), _ptr(out), _stream_ptr(stream)), "tm_orientations")
    return out


def ipf_deviation(euler_a, euler_b, laue: str, stream=None):
    """tm_ipf_deviation, Eq. (2): [B, 3] float64 radians (IPF-x, -y, -z) between
    two orientation maps. euler_a / euler_b: [B, 3] or [B, N, 3] float64
    (the first triple of each pattern is used)."""
    torch = _torch()
    if laue not in LAUE_GROUPS:
        raise ValueError(f"laue must be one of {sorted(LAUE_GROUPS)}")
    strides = []
    for name, e in (("euler_a", euler_a), ("euler_b", euler_b)):
        _require(e, name, torch.float64)
        if e.dim() not in (2, 3) or e.shape[-1] != 3:
            raise ValueError(f"{name} must be [B, 3] or [B, N, 3]")
        strides.append(3 if e.dim() == 2 else 3 * e.shape[1])
    B = euler_a.shape[0]
    if euler_b.shape[0] != B:
        raise ValueError("euler_a and euler_b must have the same number of patterns")
    out = torch.empty((B, 3), dtype=torch.float64, device=euler_a.device)
    _check(_lib.tm_ipf_deviation(_ptr(euler_a), strides[0], _ptr(euler_b), strides[1], int(B),
                                 LAUE_GROUPS[laue], _ptr(out), _stream_ptr(stream)),
           "tm_ipf_deviation")
    return out


def simulate_library(recip_basis, atoms_frac, f_atoms, g_lim: float, orientations, k: float,
                     s_max: float, g_max: float, rel_min: float = 1e-3, max_spots: int = 100,
                     stream=None, csr: bool = True):
    """tm_simulate_library: kinematical templates for orientations [T, 2]
    (Phi, phi2) radians (float64 device tensor). recip_basis [3, 3] (rows b1,
    b2, b3, 1/Angstrom), atoms_frac [n, 3] and f_atoms [n] are host arrays.
    Returns the device arrays (kx, ky, intensity [T, max_spots], count [T]),
    or with csr=True a host CSR dict (kx, ky, intensity, offsets) ready for
    Library()."""
    torch = _torch()
    Bm = np.ascontiguousarray(recip_basis, dtype=np.float64).reshape(3, 3)
    X = np.ascontiguousarray(atoms_frac, dtype=np.float64).reshape(-1, 3)
    f = np.ascontiguousarray(f_atoms, dtype=np.float64).reshape(-1)
    if len(f) != len(X):
        raise ValueError("atoms_frac and f_atoms must describe the same atoms")
    _require(orientations, "orientations", torch.float64)
    T = orientations.shape[0]
    _require(orientations, "orientations", torch.float64, (T, 2))
    dev = orientations.device
    kx = torch.empty((T, max_spots), dtype=torch.float64, device=dev)
    ky = torch.empty_like(kx)
    inten = torch.empty_like(kx)
    cnt = torch.empty((T,), dtype=torch.int32, device=dev)
    _check(_lib.tm_simulate_library(Bm.ctypes.data, X.ctypes.data, f.ctypes.data, len(f),
                                    float(g_lim), _ptr(orientations), int(T), float(k),
                                    float(s_max), float(g_max), float(rel_min), int(max_spots),
                                    _ptr(kx), _ptr(ky), _ptr(inten), _ptr(cnt),
                                    _stream_ptr(stream)), "tm_simulate_library")
    if not csr:
        return kx, ky, inten, cnt
    # host CSR for the library loader (tm_load_library reads host arrays)
    c = cnt.cpu().numpy().astype(np.int64)
    off = np.zeros(T + 1, dtype=np.int64)
    off[1:] = np.cumsum(c)
    sel = np.arange(max_spots)[None, :] < c[:, None]
    return dict(kx=kx.cpu().numpy()[sel], ky=ky.cpu().numpy()[sel],
                intensity=inten.cpu().numpy()[sel], offsets=off)


def preprocess(patterns, r_box: int = 8, frac: float = 0.5, sigma_min: float = 1.0,
               sigma_max: float = 6.0, sigma_blur: float = 1.0, threshold: float = 0.0,
               out=None, centre_out=None, stream=None):
    """tm_preprocess: direct-beam centring, difference of Gaussians, blur and
    threshold of a [B, H, W] uint16/float32 stack. Returns (float32 [B, H, W],
    float64 [B, 2] beam centres). r_box < 0, sigma_max = 0, sigma_blur = 0 and
    threshold = -inf switch the steps off."""
    torch = _torch()
    if patterns.dtype == torch.float32:
        dt = TM_F32
    elif patterns.dtype in (torch.uint16, torch.int16):
        dt = TM_U16
    else:
        raise TypeError("patterns must be float32 or uint16")
    B, H, W = patterns.shape
    _require(patterns, "patterns", patterns.dtype, (B, H, W))
    if out is None:
        out = torch.empty((B, H, W), dtype=torch.float32, device=patterns.device)
    _require(out, "out", torch.float32, (B, H, W))
    if centre_out is None:
        centre_out = torch.empty((B, 2), dtype=torch.float64, device=patterns.device)
    _require(centre_out, "centre_out", torch.float64, (B, 2))
    o = _PreOpts(int(r_box), float(frac), float(sigma_min), float(sigma_max), float(sigma_blur),
                 float(threshold))
    _check(_lib.tm_preprocess(_ptr(patterns), dt, int(B), int(H), int(W), ctypes.byref(o),
                              _ptr(out), _ptr(centre_out), _stream_ptr(stream)),
           "tm_preprocess")
    return out, centre_out


def bound_scores(lib: Library, polar, norms, stream=None):
    """tm_bound_scores: an upper bound of every template's best Q (at least
    the float32 score tm_match_batch computes) for every pattern, from
    window maxima of the polar image. Returns [B, T'] f32."""
    torch = _torch()
    B = polar.shape[0]
    compact = _layout(lib, polar)
    _require(polar, "polar", torch.float32, (B, polar.shape[1], lib.grid.n_theta))
    _require(norms, "norms", torch.float64, (B,))
    out = torch.empty((B, lib.n_total), dtype=torch.float32, device=polar.device)
    _check(_lib.tm_bound_scores(lib._h, _ptr(polar), _ptr(norms), B, compact, _ptr(out),
                                _stream_ptr(stream)), "tm_bound_scores")
    return out


def bound_scores_slots(lib: Library, polar, norms, out=None, stream=None):
    """tm_bound_scores_slots: the same bounds in the kernel's chunk-slot
    order. Returns ([B, chunks * 64] f32, slot -> template [chunks * 64]
    int32 numpy array, -1 for empty slots)."""
    torch = _torch()
    B = polar.shape[0]
    compact = _layout(lib, polar)
    _require(polar, "polar", torch.float32, (B, polar.shape[1], lib.grid.n_theta))
    _require(norms, "norms", torch.float64, (B,))
    n_cs = lib.bound_layout()["chunks"] * 64
    if out is None:
        out = torch.empty((B, n_cs), dtype=torch.float32, device=polar.device)
    _require(out, "bound_out", torch.float32, (B, n_cs))
    slots = np.empty(n_cs, dtype=np.int32)
    _check(_lib.tm_bound_scores_slots(lib._h, _ptr(polar), _ptr(norms), B, compact, _ptr(out),
                                      slots.ctypes.data, _stream_ptr(stream)),
           "tm_bound_scores_slots")
    return out, slots


def fft_scores(lib: Library, polar, norms, with_angle: bool = True, stream=None):
    """tm_fft_scores: approximate best score (and angle) of every template for
    every pattern through the Fourier route. Returns ([B, T'] f32, [B, T']
    i16 or None)."""
    torch = _torch()
    B = polar.shape[0]
    compact = _layout(lib, polar)
    _require(polar, "polar", torch.float32, (B, polar.shape[1], lib.grid.n_theta))
    _require(norms, "norms", torch.float64, (B,))
    Tn = lib.n_total
    q = torch.empty((B, Tn), dtype=torch.float32, device=polar.device)
    a = torch.empty((B, Tn), dtype=torch.int16, device=polar.device) if with_angle else None
    _check(_lib.tm_fft_scores(lib._h, _ptr(polar), _ptr(norms), B, compact, _ptr(q), _ptr(a),
                              _stream_ptr(stream)), "tm_fft_scores")
    return q, a


def topn(best_score, best_angle, N: int, stream=None):
    """tm_topn on [B, T] scores/angles. Returns (template, angle, score) [B, N]."""
    torch = _torch()
    B, T = best_score.shape
    _require(best_score, "best_score", torch.float32, (B, T))
    _require(best_angle, "best_angle", torch.int16, (B, T))
    dev = best_score.device
    tt = torch.empty((B, N), dtype=torch.int32, device=dev)
    ts = torch.empty((B, N), dtype=torch.int32, device=dev)
    tq = torch.empty((B, N), dtype=torch.float32, device=dev)
    _check(_lib.tm_topn(_ptr(best_score), _ptr(best_angle), B, T, int(N), _ptr(tt), _ptr(ts),
                        _ptr(tq), _stream_ptr(stream)), "tm_topn")
    return tt, ts, tq
