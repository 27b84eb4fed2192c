"""Masking of the dominant phase for two-stage indexing, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 4.3 (custom indexation procedures): to index nano-precipitates in a
crystalline matrix, the matrix is indexed first, then its intense
reflections are masked in every pattern, and the masked patterns are indexed
with the precipitate library. The mask is made by averaging all diffraction
patterns and thresholding the average; erosions and dilations remove small
noise-like features and make sure the tails of intense peaks are removed.
The precipitate indexation uses unit template intensities and subtracts a
small constant from the patterns (both already part of the plain path).

Readings:
* bright pixels: mean over the patterns strictly greater than the threshold;
* morphology on the bright set with the 3x3 square structuring element;
  pixels outside the image count as not bright; an opening (n_open erosions,
  then n_open dilations) removes small features, then n_grow dilations cover
  the peak tails;
* mask = 1 where the pixel is kept, 0 where it is masked;
* the mask multiplies the transformed pattern (after the gamma correction
  and the constant subtraction), so masked pixels are exactly 0: they add
  nothing to the numerator of Eq. (1) and nothing to ||P||.
"""
from __future__ import annotations

import numpy as np


def mean_pattern64(imgs: np.ndarray) -> np.ndarray:
    """Average of a stack of patterns [B, H, W] -> [H, W], float64."""
    x = np.asarray(imgs, dtype=np.float64)
    return x.sum(axis=0) / x.shape[0]


def _neighbourhood(b: np.ndarray, combine) -> np.ndarray:
    """Apply combine (all / any) over the 3x3 neighbourhood, outside = False."""
    H, W = b.shape
    p = np.zeros((H + 2, W + 2), dtype=bool)
    p[1:-1, 1:-1] = b
    stack = [p[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return combine(np.stack(stack), axis=0)


def binary_erode64(b: np.ndarray, n: int) -> np.ndarray:
    """n erosions: a pixel stays set iff its whole 3x3 neighbourhood is set."""
    b = np.asarray(b, dtype=bool)
    for _ in range(n):
        b = _neighbourhood(b, np.all)
    return b


def binary_dilate64(b: np.ndarray, n: int) -> np.ndarray:
    """n dilations: a pixel becomes set iff any pixel of its 3x3
    neighbourhood is set."""
    b = np.asarray(b, dtype=bool)
    for _ in range(n):
        b = _neighbourhood(b, np.any)
    return b


def matrix_mask64(imgs: np.ndarray, threshold: float, n_open: int = 1,
                  n_grow: int = 2) -> np.ndarray:
    """Mask [H, W] float64 (1 keep, 0 masked) of the reflections that are
    bright in the average pattern."""
    bright = mean_pattern64(imgs) > threshold
    bright = binary_dilate64(binary_erode64(bright, n_open), n_open)
    bright = binary_dilate64(bright, n_grow)
    return np.where(bright, 0.0, 1.0)
