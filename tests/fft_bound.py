"""A-priori error bound of the FP16 Fourier-route scorer (test helper).

The GPU library reports the bound it certifies with; this module derives the
same quantity independently, so the tests can (a) check it against an exact
emulation of the reduced-precision arithmetic on the CPU and (b) check that
the library's value agrees.

Arithmetic being bounded (every quantity normalised so that the exact score
is Q(s) = (1/n) sum_k c_k Re(C(k) e^{2 pi i k s / n}), n = n_theta, c_k = 1 at
k = 0 and k = n/2, else 2):

* template spectra T[j, k] of the weights divided by ||T||, computed in
  float64, scaled by 2^8 and rounded once to float16;
* pattern spectra P[j, k] of the polar rows divided by ||P||, computed in
  float64, scaled by 2^8, rounded to float32 and then to float16;
* C(k) = sum_j conj(T) P accumulated in float32 over the R rows, rescaled
  by a power of two 2^sc and rounded to float16;
* the inverse transform with float16 cosine / sine tables scaled by 2^12,
  accumulated in float32 over the frequencies, then one addition and one
  scaling in float32;
* plus the exact rescoring path's own float32 error, so that the margin
  covers |Q_fft - Q_fp32| for every template and shift.

A float16 value below the smallest normal number may be flushed to zero; the
bound allows an absolute error of 2^-14 (in scaled units) on every rounding.
Parseval's identity turns the per-element relative errors into a bound on Q:
(1/n) ||X||_c ||Y||_c <= 1 for the exact normalised spectra.
"""
from __future__ import annotations

import math

U16 = 2.0 ** -11
U32 = 2.0 ** -24
TINY16 = 2.0 ** -14
SCALE_T = 8
SCALE_P = 8
SCALE_W = 12


def gamma32(n: int) -> float:
    return n * U32 / (1.0 - n * U32)


def freq_padded(n_theta: int) -> int:
    """Frequencies k = 0..n/2, padded to a multiple of 16."""
    F = n_theta // 2 + 1
    return (F + 15) // 16 * 16


def spectrum_scale(n_row_max: int, n_theta: int) -> int:
    """Power of two applied to C(k) before float16 storage: |C(k)| <=
    sqrt(n_row_max * n) after normalisation, kept below 2^15."""
    m = math.sqrt(max(1, n_row_max) * n_theta)
    return int(math.floor(math.log2(32768.0 / m)))


def fft16_error_bound(R: int, n_theta: int, n_row_max: int, n_max: int) -> float:
    sc = spectrum_scale(n_row_max, n_theta)
    eT = TINY16 * 2.0 ** -SCALE_T
    eP = TINY16 * 2.0 ** -SCALE_P
    eC = TINY16 * 2.0 ** -sc
    eW = TINY16 * 2.0 ** -SCALE_W
    r2 = math.sqrt(2.0)
    aT = U16 + r2 * eT * math.sqrt(R)
    aP = U16 + 2 * U32 + r2 * eP * math.sqrt(R)
    e1 = aT + aP + aT * aP                      # rounded input spectra
    rho2 = (1.0 + aT) * (1.0 + aP)
    gf = gamma32(R + 2)
    e2 = 2.0 * gf * rho2                        # forward accumulation
    m0 = (1.0 + 2.0 * gf) * rho2
    e3 = U16 * m0 + r2 * eC                     # float16 storage of C(k)
    m = (1.0 + U16) * m0 + r2 * eC
    gi = gamma32(freq_padded(n_theta) + 1)
    e4 = (U16 + r2 * eW) * m + gi * (1.0 + U16 + r2 * eW) * m   # inverse
    e5 = 3.0 * U32 * (m + e4)                   # final add and scaling
    d32 = gamma32(n_max + 3)                    # exact float32 rescoring
    return e1 + e2 + e3 + e4 + e5 + d32 + 1e-9
