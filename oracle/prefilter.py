"""Library pre-filter by azimuthally integrated profiles, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 2.2 (Fig. 3): the image and the templates are integrated over the
azimuthal direction; the correlation between the integrated image and the
integrated library is one matrix-vector product; only the best-correlating
templates (typically a tenth) go on to the full in-plane search.

Readings:
* image profile prof_P[j] = sum_k P[j, k]; template profile prof_T[t, j] = sum
  of the merged pixel weights of base template t in row j (a mirror has the
  same profile as its base);
* the correlation is the cosine of the two profiles (0 if either is zero);
* keep the first ceil(f * T) base templates ordered by (-cosine, t), plus
  their mirrors; f = 0.1 by default;
* the kept templates are then scored exactly as in the plain path.
"""
from __future__ import annotations

import math

import numpy as np

from .library import OracleLibrary
from .match import match_exact64, topn64
from .polar import norm64, polar64, profile64


def radial_profiles64(lib: OracleLibrary) -> np.ndarray:
    """prof_T [T_base, R]: per base template, summed weights per polar row."""
    Tb = lib.T_base
    prof = np.zeros((Tb, lib.R), dtype=np.float64)
    base = lib.tid < Tb
    np.add.at(prof, (lib.tid[base], lib.J[base]), lib.Wt[base])
    return prof


def prefilter64(prof_P: np.ndarray, prof_T: np.ndarray, keep: float):
    """Base templates kept by the pre-filter (ascending order of rank) and
    the cosine scores [T_base]."""
    prof_P = np.asarray(prof_P, dtype=np.float64)
    dots = prof_T @ prof_P                       # the single matrix-vector product
    den = np.linalg.norm(prof_T, axis=1) * np.linalg.norm(prof_P)
    cos = np.zeros(len(prof_T), dtype=np.float64)
    ok = den > 0.0
    cos[ok] = dots[ok] / den[ok]
    n_keep = min(len(prof_T), int(math.ceil(keep * len(prof_T))))
    order = np.lexsort((np.arange(len(prof_T)), -cos))[:n_keep]
    return order.astype(np.int64), cos


def index_pattern_prefiltered64(img: np.ndarray, lib: OracleLibrary, N: int, keep: float = 0.1,
                                mirror=True, r0=0.0, dr=1.0, cx=None, cy=None, gamma=1.0,
                                subtract=0.0, interp="bilinear", prof_T=None):
    """Pre-filtered path for one pattern: kept base templates (and mirrors)
    scored exactly, top-N among them. Returns (t, s, Q, kept_ids)."""
    P = polar64(img, lib.R, lib.n_theta, r0, dr, cx, cy, gamma, subtract, interp)
    pn = norm64(P)
    prof_T = radial_profiles64(lib) if prof_T is None else prof_T
    kept, _ = prefilter64(profile64(P), prof_T, keep)
    ids = np.concatenate([kept, kept + lib.T_base]) if mirror else kept
    ids = np.sort(ids)
    sub = lib.subset(ids)
    best, arg = match_exact64(P, sub, pn)
    t, s, q = topn64(best, arg, N, templates=ids)
    return t, s, q, ids
