"""Polar resampling of a diffraction pattern, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 2.2: the image is converted to polar coordinates about the centre of
the direct beam; the width of the polar image fixes the in-plane angular step
(360 degrees divided by the number of columns, so 360 columns give 1 degree).

Readings (the paper does not specify these):
* sample radii r_j = r0 + j*dr for j in [0, R), angles theta_k = 2*pi*k/n_theta
  for k in [0, n_theta), measured from +x (image columns) toward +y (image
  rows);
* the image is indexed img[y, x] and pixel (row i, column j) sits at
  (x = j, y = i); the sample point of (j, k) is (cx + r_j cos theta_k,
  cy + r_j sin theta_k);
* interpolation is bilinear with zero padding outside the image (nearest
  neighbour as an option);
* the intensity transform is applied to the Cartesian pixels before
  resampling: clamp at zero and raise to gamma when gamma != 1, then subtract
  a constant.
"""
from __future__ import annotations

import numpy as np


def polar_coords64(R: int, n_theta: int, r0: float, dr: float, cx: float, cy: float):
    """Sample coordinates (x, y), each [R, n_theta] float64."""
    r = r0 + dr * np.arange(R, dtype=np.float64)
    th = 2.0 * np.pi * np.arange(n_theta, dtype=np.float64) / n_theta
    x = cx + r[:, None] * np.cos(th)[None, :]
    y = cy + r[:, None] * np.sin(th)[None, :]
    return x, y


def intensity_transform64(img: np.ndarray, gamma: float = 1.0, subtract: float = 0.0) -> np.ndarray:
    """Gamma correction (power < 1 boosts weak reflections) then subtraction
    of a constant (penalises template spots that fall on background),
    Section 2.2. Identity for gamma = 1, subtract = 0."""
    x = np.asarray(img, dtype=np.float64)
    if gamma != 1.0:
        x = np.power(np.maximum(x, 0.0), gamma)
    return x - subtract


def _pixel(img: np.ndarray, yi: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """img[yi, xi] with zero outside the image."""
    H, W = img.shape
    ok = (yi >= 0) & (yi < H) & (xi >= 0) & (xi < W)
    out = np.zeros(yi.shape, dtype=np.float64)
    out[ok] = img[yi[ok], xi[ok]]
    return out


def bilinear64(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of img at (x, y) with zero padding."""
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    xi = x0.astype(np.int64)
    yi = y0.astype(np.int64)
    p00 = _pixel(img, yi, xi)
    p01 = _pixel(img, yi, xi + 1)
    p10 = _pixel(img, yi + 1, xi)
    p11 = _pixel(img, yi + 1, xi + 1)
    return ((1.0 - fx) * (1.0 - fy) * p00 + fx * (1.0 - fy) * p01
            + (1.0 - fx) * fy * p10 + fx * fy * p11)


def nearest64(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    return _pixel(img, np.rint(y).astype(np.int64), np.rint(x).astype(np.int64))


def polar64(img: np.ndarray, R: int, n_theta: int, r0: float = 0.0, dr: float = 1.0,
            cx: float | None = None, cy: float | None = None, gamma: float = 1.0,
            subtract: float = 0.0, interp: str = "bilinear", mask=None) -> np.ndarray:
    """Polar image P[j, k] of one pattern, float64 [R, n_theta]. An optional
    [H, W] mask multiplies the transformed pattern before resampling (the
    masking step of two-stage indexing, Section 4; see oracle.mask)."""
    H, W = img.shape
    cx = W / 2.0 if cx is None else cx
    cy = H / 2.0 if cy is None else cy
    t = intensity_transform64(img, gamma, subtract)
    if mask is not None:
        t = t * np.asarray(mask, dtype=np.float64)
    x, y = polar_coords64(R, n_theta, r0, dr, cx, cy)
    if interp == "bilinear":
        return bilinear64(t, x, y)
    if interp == "nearest":
        return nearest64(t, x, y)
    raise ValueError(interp)


def norm64(P: np.ndarray) -> float:
    """||P|| over all polar pixels (Eq. 1 denominator, image factor)."""
    return float(np.sqrt(np.sum(np.asarray(P, dtype=np.float64) ** 2)))


def profile64(P: np.ndarray) -> np.ndarray:
    """Azimuthal integral of the polar image, one value per radius (Fig. 3)."""
    return np.asarray(P, dtype=np.float64).sum(axis=1)
