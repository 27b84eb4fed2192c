"""Pattern preprocessing before indexing, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 4.1 lists the preprocessing applied before template matching: the
direct beam of every pattern is centred, the diffuse background is removed
by a difference of Gaussians, the result is smoothed by a Gaussian blur, and
low-intensity pixels are set to zero (the gamma correction that follows is
the intensity transform of the polar step). The discussion names
parallelising these steps as an open optimisation.

Readings:
* beam centre: the intensity-weighted centroid of the pixels within the
  square box |x - W/2| <= r_box, |y - H/2| <= r_box (pixel-index
  coordinates, x = column) whose value is >= frac times the box's maximum;
  a box whose maximum is <= 0 leaves the pattern where it is;
* centring: out(x, y) = in(x + cx - W/2, y + cy - H/2), bilinear, zero
  outside the image, so the beam lands on (W/2, H/2), the polar grid's
  default origin;
* Gaussian filter: separable, sampled Gaussian exp(-t^2 / (2 sigma^2)) on
  |t| <= floor(4 sigma + 0.5), normalised to sum 1, mirror boundary
  (... c b a | a b c ...), rows (along x) first, then columns; sigma = 0
  leaves the image unchanged;
* difference of Gaussians: G(sigma_min) - G(sigma_max) of the centred image
  (sigma_min < sigma_max; G(0) is the identity); blur: G(sigma_blur) of
  that; threshold: values < threshold become 0.
"""
from __future__ import annotations

import numpy as np


def gaussian_weights64(sigma: float) -> np.ndarray:
    """Normalised sampled Gaussian on [-r, r], r = floor(4 sigma + 0.5)."""
    if sigma <= 0.0:
        return np.ones(1)
    r = int(4.0 * sigma + 0.5)
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-t * t / (2.0 * sigma * sigma))
    return w / w.sum()


def convolve_axis64(img: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """Correlation with the symmetric weights w along one axis, mirror
    boundary: each output is sum_t w[t + r] * in[mirror(i + t)]."""
    img = np.asarray(img, dtype=np.float64)
    r = (len(w) - 1) // 2
    n = img.shape[axis]
    out = np.zeros_like(img)
    for t in range(-r, r + 1):
        idx = np.arange(n) + t
        # mirror about the edges (edge sample repeated), folded until in range
        while np.any((idx < 0) | (idx >= n)):
            idx = np.where(idx < 0, -idx - 1, idx)
            idx = np.where(idx >= n, 2 * n - idx - 1, idx)
        out += w[t + r] * np.take(img, idx, axis=axis)
    return out


def gaussian64(img: np.ndarray, sigma: float) -> np.ndarray:
    w = gaussian_weights64(sigma)
    return convolve_axis64(convolve_axis64(img, w, axis=1), w, axis=0)


def beam_centre64(img: np.ndarray, r_box: int, frac: float):
    """(cx, cy) of the direct beam (see the module readings)."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x0, y0 = W / 2.0, H / 2.0
    xs = [x for x in range(W) if abs(x - x0) <= r_box]
    ys = [y for y in range(H) if abs(y - y0) <= r_box]
    box = img[np.ix_(ys, xs)]
    m = box.max() if box.size else 0.0
    if not m > 0.0:
        return x0, y0
    sel = box >= frac * m
    v = box * sel
    X, Y = np.meshgrid(np.array(xs, dtype=np.float64), np.array(ys, dtype=np.float64))
    s = v.sum()
    return float((v * X).sum() / s), float((v * Y).sum() / s)


def shift_image64(img: np.ndarray, dx: float, dy: float) -> np.ndarray:
    """out(x, y) = in(x + dx, y + dy), bilinear, zero outside."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    xs, ys = X + dx, Y + dy
    x0, y0 = np.floor(xs), np.floor(ys)
    fx, fy = xs - x0, ys - y0
    xi, yi = x0.astype(np.int64), y0.astype(np.int64)

    def px(yy, xx):
        ok = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H)
        return np.where(ok, img[np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1)], 0.0)
    return ((1 - fx) * (1 - fy) * px(yi, xi) + fx * (1 - fy) * px(yi, xi + 1)
            + (1 - fx) * fy * px(yi + 1, xi) + fx * fy * px(yi + 1, xi + 1))


def preprocess64(img: np.ndarray, r_box: int = 8, frac: float = 0.5, sigma_min: float = 1.0,
                 sigma_max: float = 6.0, sigma_blur: float = 1.0, threshold: float = 0.0):
    """The four steps in the paper's order; returns (image, (cx, cy)).
    r_box < 0 skips the centring, sigma_max = 0 the difference of Gaussians,
    sigma_blur = 0 the blur, threshold = -inf the threshold."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    if r_box >= 0:
        cx, cy = beam_centre64(img, r_box, frac)
        c = shift_image64(img, cx - W / 2.0, cy - H / 2.0)
    else:
        cx, cy = W / 2.0, H / 2.0
        c = img
    d = gaussian64(c, sigma_min) - gaussian64(c, sigma_max) if sigma_max > 0 else c
    b = gaussian64(d, sigma_blur)
    return np.where(b < threshold, 0.0, b), (cx, cy)
