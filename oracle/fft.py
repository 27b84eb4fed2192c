"""In-plane search through Fourier transforms along the azimuth, in float64
(oracle).

Test infrastructure only (see the package docstring).

Section 2.2 (computational cost): sliding a template along the azimuthal axis
of the polar image with wraparound is a circular cross-correlation along
theta, so it can be evaluated with fast Fourier transforms at a cost that
grows as r * phi * log(phi) instead of with the number of spots; the paper
notes this pays off only for templates with very many spots on its CPU.

What is computed here is the same correlation index as the direct search,
reached through the correlation theorem:

    numerator(t, s) = sum_j sum_theta T_t[j, theta] P[j, theta + s]
                    = irfft( sum_j conj(rfft T_t[j]) * rfft P[j] )[s]

with T_t the dense [R, n_theta] image of template t's merged pixel weights.
It equals the direct numerator exactly in exact arithmetic.

Readings:
* real DFT along theta with frequencies k = 0 .. n_theta // 2 and the inverse
  scaled by 1 / n_theta (numpy's rfft / irfft conventions);
* mirrors use their own reflected pixels (k -> -k), so their spectra are the
  complex conjugates of the base spectra; nothing else changes;
* scores are normalised exactly as in Eq. (1); Q = 0 when a norm is zero;
  per template the best shift is the smallest maximising s.
"""
from __future__ import annotations

import numpy as np

from .library import OracleLibrary
from .polar import norm64


def template_images64(lib: OracleLibrary, t_lo: int, t_hi: int) -> np.ndarray:
    """Dense polar images [t_hi - t_lo, R, n_theta] of the merged template
    pixels (weights, unnormalised)."""
    D = np.zeros((t_hi - t_lo, lib.R, lib.n_theta), dtype=np.float64)
    a, b = lib.starts[t_lo], lib.starts[t_hi]
    np.add.at(D, (lib.tid[a:b] - t_lo, lib.J[a:b], lib.K[a:b]), lib.Wt[a:b])
    return D


def fft_numerators64(P: np.ndarray, lib: OracleLibrary, t_lo: int, t_hi: int) -> np.ndarray:
    """Numerators C[t, s] for templates [t_lo, t_hi) by the correlation
    theorem along theta."""
    P = np.asarray(P, dtype=np.float64)
    n_theta = P.shape[1]
    Ph = np.fft.rfft(P, axis=1)                                   # [R, F]
    Th = np.fft.rfft(template_images64(lib, t_lo, t_hi), axis=2)  # [c, R, F]
    spec = np.einsum("crk,rk->ck", np.conj(Th), Ph)               # sum over rows j
    return np.fft.irfft(spec, n=n_theta, axis=1)


def fft_match64(P: np.ndarray, lib: OracleLibrary, pnorm: float | None = None,
                chunk: int = 256):
    """Best Q and its smallest maximising shift for every template, through
    the Fourier route: ([T'], [T'])."""
    P = np.asarray(P, dtype=np.float64)
    pnorm = norm64(P) if pnorm is None else pnorm
    Tn = lib.n_total
    best = np.zeros(Tn, dtype=np.float64)
    arg = np.zeros(Tn, dtype=np.int64)
    for lo in range(0, Tn, chunk):
        hi = min(Tn, lo + chunk)
        C = fft_numerators64(P, lib, lo, hi)
        den = pnorm * lib.tnorm[lo:hi]
        Q = np.zeros_like(C)
        ok = den > 0.0
        Q[ok] = C[ok] / den[ok, None]
        arg[lo:hi] = np.argmax(Q, axis=1)
        best[lo:hi] = Q[np.arange(hi - lo), arg[lo:hi]]
    return best, arg
