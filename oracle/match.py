"""Correlation index, in-plane search and top-N, in float64 (oracle).

Test infrastructure only (see the package docstring).

Eq. (1): Q = sum_i P(x_i, y_i) T(x_i, y_i) / (sqrt(sum_i P^2) sqrt(sum_i T^2)).
The template is non-zero only at its spots, so the numerator is a sum over
template pixels. Section 2.2: the template is slid along the azimuthal axis
with wraparound and Q is evaluated at every shift; the maximum and the angle
where it occurs are kept per template; the pattern is indexed by the template
with the highest Q, or by the N best after sorting.

Readings:
* Q(t, s) = sum_{(j,k,w) in t} w * P[j, (k + s) mod n_theta] / (||P|| ||T_t||)
  for s in [0, n_theta); the shift s is the counter-clockwise rotation (in the
  +x -> +y sense) that takes the template onto the pattern; in degrees it is
  s * 360 / n_theta;
* Q = 0 when either norm is zero;
* per template the best shift is the smallest maximising s;
* top-N: N distinct templates ordered by Q descending, ties by lower template
  index (mirrors have indices T..2T-1).
"""
from __future__ import annotations

import numpy as np

from .library import OracleLibrary
from .polar import norm64, polar64


def _numerators(P: np.ndarray, lib: OracleLibrary, t_lo: int, t_hi: int) -> np.ndarray:
    """Eq. (1) numerators C[t, s] for templates [t_lo, t_hi), float64."""
    n_theta = P.shape[1]
    a, b = lib.starts[t_lo], lib.starts[t_hi]
    s = np.arange(n_theta)
    out = np.zeros((t_hi - t_lo, n_theta), dtype=np.float64)
    if b == a:
        return out
    J = lib.J[a:b]
    K = lib.K[a:b]
    g = P[J[:, None], (K[:, None] + s[None, :]) % n_theta] * lib.Wt[a:b, None]
    # sum each template's pixel contributions (templates are contiguous)
    seg = lib.starts[t_lo:t_hi] - a
    nonempty = np.diff(lib.starts[t_lo:t_hi + 1]) > 0
    if nonempty.any():
        out[nonempty] = np.add.reduceat(g, seg[nonempty], axis=0)
    return out


def scores64(P: np.ndarray, lib: OracleLibrary, pnorm: float | None = None) -> np.ndarray:
    """Full Q tensor [T', n_theta] for one polar image (small cases)."""
    P = np.asarray(P, dtype=np.float64)
    pnorm = norm64(P) if pnorm is None else pnorm
    C = _numerators(P, lib, 0, lib.n_total)
    den = pnorm * lib.tnorm
    Q = np.zeros_like(C)
    ok = den > 0.0
    Q[ok] = C[ok] / den[ok, None]
    return Q


def match_exact64(P: np.ndarray, lib: OracleLibrary, pnorm: float | None = None,
                  chunk: int = 512):
    """Best Q and its (smallest) shift for every template: ([T'], [T'])."""
    P = np.asarray(P, dtype=np.float64)
    pnorm = norm64(P) if pnorm is None else pnorm
    Tn = lib.n_total
    best = np.zeros(Tn, dtype=np.float64)
    arg = np.zeros(Tn, dtype=np.int64)
    for lo in range(0, Tn, chunk):
        hi = min(Tn, lo + chunk)
        C = _numerators(P, lib, lo, hi)
        den = pnorm * lib.tnorm[lo:hi]
        Q = np.zeros_like(C)
        ok = den > 0.0
        Q[ok] = C[ok] / den[ok, None]
        arg[lo:hi] = np.argmax(Q, axis=1)          # first maximum
        best[lo:hi] = Q[np.arange(hi - lo), arg[lo:hi]]
    return best, arg


def topn64(best: np.ndarray, arg: np.ndarray, N: int, templates=None):
    """N best (template, shift, Q) by Q descending, ties by lower template
    index. ``templates`` maps positions of best/arg to template ids."""
    best = np.asarray(best, dtype=np.float64)
    tids = np.arange(len(best)) if templates is None else np.asarray(templates)
    order = np.lexsort((tids, -best))[:N]
    return tids[order].astype(np.int64), np.asarray(arg)[order].astype(np.int64), best[order]


def index_pattern64(img: np.ndarray, lib: OracleLibrary, N: int, r0=0.0, dr=1.0,
                    cx=None, cy=None, gamma=1.0, subtract=0.0, interp="bilinear"):
    """Whole plain path for one pattern: polar image, Q at every shift for
    every template, top-N. Returns (t [N], s [N], Q [N], ||P||)."""
    P = polar64(img, lib.R, lib.n_theta, r0, dr, cx, cy, gamma, subtract, interp)
    pn = norm64(P)
    best, arg = match_exact64(P, lib, pn)
    t, s, q = topn64(best, arg, N)
    return t, s, q, pn


def _index_one(args):
    img, lib, N, kw = args
    return index_pattern64(img, lib, N, **kw)


def index_batch64(imgs: np.ndarray, lib: OracleLibrary, N: int, processes: int = 1, **kw):
    """index_pattern64 over a stack of patterns; optional process pool."""
    jobs = [(imgs[i], lib, N, kw) for i in range(len(imgs))]
    if processes <= 1:
        res = [_index_one(j) for j in jobs]
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            res = pool.map(_index_one, jobs, chunksize=1)
    t = np.stack([r[0] for r in res])
    s = np.stack([r[1] for r in res])
    q = np.stack([r[2] for r in res])
    pn = np.array([r[3] for r in res])
    return t, s, q, pn


def refine_angle64(P: np.ndarray, lib: OracleLibrary, t: int, s: int,
                   pnorm: float | None = None) -> float:
    """Sub-bin in-plane angle of template t around its best shift s
    (Section 5, discussion: improving the optimisation of the in-plane angle).

    Reading: the parabola through Q(t, s-1), Q(t, s), Q(t, s+1) (shifts mod
    n_theta); its vertex offset d = (q- - q+) / (2 (q- - 2 q0 + q+)) is used
    when the curvature q- - 2 q0 + q+ is negative (a maximum), clipped to
    [-1/2, 1/2], else d = 0. Returns (s + d) * 360 / n_theta in degrees,
    taken modulo 360."""
    n_theta = lib.n_theta
    Q = scores64(P, lib.subset([int(t)]), pnorm)[0]
    qm, q0, qp = Q[(s - 1) % n_theta], Q[s % n_theta], Q[(s + 1) % n_theta]
    den = qm - 2.0 * q0 + qp
    d = 0.0
    if den < 0.0:
        d = min(0.5, max(-0.5, 0.5 * (qm - qp) / den))
    return float(((s + d) * 360.0 / n_theta) % 360.0)
