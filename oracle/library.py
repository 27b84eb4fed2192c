"""Template spots to integer polar pixels, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 2.1: a template is a list of Bragg spots (kx, ky)_i with intensity
I_i. Section 2.2: the polar coordinates (r_i, phi_i') of the spots are rounded
to the nearest integer so they address pixels of the polar image; mirror
templates are obtained by reflecting the spots across y = 0 and must be
considered alongside the originals.

Readings:
* rho = px_per_inv_A * hypot(kx, ky); j = rint((rho - r0)/dr);
  k = rint(atan2(ky, kx) * n_theta / (2 pi)) mod n_theta; rint is
  round-half-to-even;
* spots with j outside [0, R) are dropped; the direct beam (0, 0) is dropped
  unless keep_direct_beam;
* spots of one template that round to the same pixel are merged by summing
  their weights, so Eq. (1) holds literally over pixels;
* weight = intensity, or 1 with unit intensities (Section 4.3);
* template indices: base templates 0..T-1, mirror of t is T + t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _spot_pixels(kx, ky, w, px_per, R, n_theta, r0, dr, keep_direct_beam):
    kx = np.asarray(kx, dtype=np.float64)
    ky = np.asarray(ky, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    keep = np.ones(len(kx), dtype=bool)
    if not keep_direct_beam:
        keep &= ~((kx == 0.0) & (ky == 0.0))
    rho = px_per * np.hypot(kx, ky)
    j = np.rint((rho - r0) / dr)
    k = np.mod(np.rint(np.arctan2(ky, kx) * n_theta / (2.0 * np.pi)), n_theta)
    keep &= (j >= 0) & (j < R)
    j = j[keep].astype(np.int64)
    k = k[keep].astype(np.int64)
    w = w[keep]
    # merge spots falling on the same polar pixel by summing their weights
    key = j * n_theta + k
    uk, inv = np.unique(key, return_inverse=True)
    wm = np.bincount(inv, weights=w, minlength=len(uk))
    return (uk // n_theta).astype(np.int64), (uk % n_theta).astype(np.int64), wm


def template_pixels64(kx, ky, intensity, offsets, px_per, R, n_theta, r0=0.0, dr=1.0,
                      mirror=True, unit=False, keep_direct_beam=False):
    """Per-template merged polar pixels.

    Returns a list of (j, k, w) arrays, T entries, or 2T with mirrors (the
    mirror of base t is entry T + t, computed by literally reflecting the
    spots across y = 0 and converting again)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    T = len(offsets) - 1
    out = []
    for sign in ((1.0, -1.0) if mirror else (1.0,)):
        for t in range(T):
            a, b = offsets[t], offsets[t + 1]
            w = np.ones(b - a) if unit else np.asarray(intensity[a:b], dtype=np.float64)
            out.append(_spot_pixels(kx[a:b], sign * np.asarray(ky[a:b], dtype=np.float64),
                                    w, px_per, R, n_theta, r0, dr, keep_direct_beam))
    return out


@dataclass
class OracleLibrary:
    """Flattened oracle library: every merged pixel of every template (base
    then mirrors), with its template id, and the template norms ||T||."""
    R: int
    n_theta: int
    T_base: int
    J: np.ndarray
    K: np.ndarray
    Wt: np.ndarray
    tid: np.ndarray
    starts: np.ndarray      # [T'+1]
    tnorm: np.ndarray       # [T']

    @property
    def n_total(self) -> int:
        return len(self.starts) - 1

    @classmethod
    def build(cls, lib: dict, px_per: float, R: int, n_theta: int, r0=0.0, dr=1.0,
              mirror=True, unit=False, keep_direct_beam=False):
        pix = template_pixels64(lib["kx"], lib["ky"], lib["intensity"], lib["offsets"],
                                px_per, R, n_theta, r0, dr, mirror, unit, keep_direct_beam)
        counts = np.array([len(p[0]) for p in pix], dtype=np.int64)
        starts = np.zeros(len(pix) + 1, dtype=np.int64)
        starts[1:] = np.cumsum(counts)
        J = np.concatenate([p[0] for p in pix]) if pix else np.zeros(0, np.int64)
        K = np.concatenate([p[1] for p in pix]) if pix else np.zeros(0, np.int64)
        Wt = np.concatenate([p[2] for p in pix]) if pix else np.zeros(0)
        tid = np.repeat(np.arange(len(pix)), counts)
        # ||T|| = sqrt(sum of squared pixel weights), Eq. (1)
        tnorm = np.sqrt(np.bincount(tid, weights=Wt * Wt, minlength=len(pix)))
        return cls(R, n_theta, len(lib["offsets"]) - 1, J, K, Wt, tid, starts, tnorm)

    def subset(self, templates) -> "OracleLibrary":
        """Library restricted to the given template ids (kept in the given
        order; the caller maps local indices back)."""
        templates = np.asarray(templates, dtype=np.int64)
        parts = [np.arange(self.starts[t], self.starts[t + 1]) for t in templates]
        sel = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        counts = self.starts[templates + 1] - self.starts[templates]
        starts = np.zeros(len(templates) + 1, dtype=np.int64)
        starts[1:] = np.cumsum(counts)
        tid = np.repeat(np.arange(len(templates)), counts)
        return OracleLibrary(self.R, self.n_theta, self.T_base, self.J[sel], self.K[sel],
                             self.Wt[sel], tid, starts, self.tnorm[templates])
