"""Kinematical simulation of template libraries, in float64 (oracle).

Test infrastructure only (see the package docstring).

Section 2.1 builds each template in four steps:
1. the reciprocal lattice points up to a maximum radius;
2. the grid rotated by the orientation (phi1 = 0, Phi, phi2), and each
   point's distance to the surface of the Ewald sphere (the excitation
   error);
3. the spot intensity: I = F F* (structure factor) times a shape factor of
   the excitation error (the relrods); atomic scattering factors may be set
   to 1 (the option the paper recommends for template matching);
4. the spots close to the Ewald sphere projected onto the kx-ky plane, the
   rest discarded.

Readings:
* grid: all hkl != 000 with |g| <= g_lim, g = h b1 + k b2 + l b3 (reciprocal
  basis rows, 1/Angstrom, no 2 pi), in lexicographic (h, k, l) order;
  reflections with F F* <= 1e-6 (systematic absences) are dropped;
* structure factor F = sum_atoms f_a exp(2 pi i (h x + k y + l z)) with one
  constant f_a per atom (1 for unit scattering factors);
* the orientation rotates crystal vectors into the sample frame with
  g^T, g the Bunge matrix of (0, Phi, phi2) (the frame of the orientation
  output);
* incident beam along -z, wave number k = 1/lambda: the Ewald sphere has its
  centre at (0, 0, k) and passes through the origin; excitation error
  s = k - |g - (0, 0, k)| (positive inside the sphere);
* shape factor: linear relrod of half-width s_max, max(0, 1 - |s| / s_max);
* a spot is kept if its shape factor is positive and its projected radius
  sqrt(gx^2 + gy^2) <= g_max; then spots below rel_min times the template's
  brightest are dropped, the rest ordered by intensity (descending, ties in
  grid order), cut to max_spots, and intensities divided by the brightest.
"""
from __future__ import annotations

import numpy as np

from .orient import bunge_matrix64


def reciprocal_grid64(recip_basis, g_lim: float):
    """hkl [n, 3] int64 and g [n, 3] float64 of every grid point with
    0 < |g| <= g_lim, lexicographic in (h, k, l)."""
    Bm = np.asarray(recip_basis, dtype=np.float64)
    A = np.linalg.inv(Bm).T                      # real-space basis: a_i . b_j = delta_ij
    # |h_i| = |g . a_i| <= |g| |a_i|
    lim = [int(np.floor(g_lim * np.linalg.norm(A[i]) + 1e-9)) for i in range(3)]
    rows = []
    for h in range(-lim[0], lim[0] + 1):
        for k in range(-lim[1], lim[1] + 1):
            for l in range(-lim[2], lim[2] + 1):
                if h == 0 and k == 0 and l == 0:
                    continue
                g = h * Bm[0] + k * Bm[1] + l * Bm[2]
                if np.sqrt(g @ g) <= g_lim:
                    rows.append((h, k, l))
    hkl = np.array(rows, dtype=np.int64).reshape(-1, 3)
    return hkl, hkl.astype(np.float64) @ Bm


def structure_factor_sq64(hkl, atoms_frac, f_atoms) -> np.ndarray:
    """F F* for each hkl (Section 2.1)."""
    hkl = np.asarray(hkl, dtype=np.float64)
    x = np.asarray(atoms_frac, dtype=np.float64).reshape(-1, 3)
    f = np.asarray(f_atoms, dtype=np.float64).reshape(-1)
    F = np.zeros(len(hkl), dtype=np.complex128)
    for a in range(len(x)):
        F += f[a] * np.exp(2j * np.pi * (hkl @ x[a]))
    return (F * np.conj(F)).real


def reflections64(recip_basis, atoms_frac, f_atoms, g_lim: float):
    """The grid of step 1 without systematic absences: (hkl, g, F F*)."""
    hkl, g = reciprocal_grid64(recip_basis, g_lim)
    F2 = structure_factor_sq64(hkl, atoms_frac, f_atoms)
    keep = F2 > 1e-6
    return hkl[keep], g[keep], F2[keep]


def excitation_error64(g_sample: np.ndarray, k: float) -> np.ndarray:
    """Distance to the Ewald sphere surface, positive inside (step 2)."""
    d = g_sample - np.array([0.0, 0.0, k])
    return k - np.sqrt(np.sum(d * d, axis=-1))


def shape_factor64(s: np.ndarray, s_max: float) -> np.ndarray:
    """Linear relrod profile (step 3)."""
    return np.maximum(0.0, 1.0 - np.abs(s) / s_max)


def simulate_template64(g_c, F2, Phi: float, phi2: float, k: float, s_max: float,
                        g_max: float, rel_min: float, max_spots: int):
    """One template (steps 2-4): spots (kx, ky) in 1/Angstrom and relative
    intensities, brightest first."""
    M = bunge_matrix64(0.0, Phi, phi2).T          # crystal -> sample
    gs = np.asarray(g_c, dtype=np.float64) @ M.T
    shape = shape_factor64(excitation_error64(gs, k), s_max)
    I = np.asarray(F2, dtype=np.float64) * shape
    ok = (shape > 0.0) & (np.hypot(gs[:, 0], gs[:, 1]) <= g_max)
    idx = np.nonzero(ok)[0]
    if len(idx) == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    top = I[idx].max()
    idx = idx[I[idx] >= rel_min * top]
    order = sorted(idx.tolist(), key=lambda i: (-I[i], i))[:max_spots]
    order = np.array(order, dtype=np.int64)
    return gs[order, 0], gs[order, 1], I[order] / top


def simulate_library64(recip_basis, atoms_frac, f_atoms, g_lim, orientations, k, s_max,
                       g_max, rel_min, max_spots):
    """CSR library (kx, ky, intensity, offsets) for orientations [T, 2]
    = (Phi, phi2)."""
    _, g_c, F2 = reflections64(recip_basis, atoms_frac, f_atoms, g_lim)
    kx, ky, I, off = [], [], [], [0]
    for Phi, phi2 in np.asarray(orientations, dtype=np.float64).reshape(-1, 2):
        a, b, c = simulate_template64(g_c, F2, Phi, phi2, k, s_max, g_max, rel_min, max_spots)
        kx.append(a)
        ky.append(b)
        I.append(c)
        off.append(off[-1] + len(a))
    cat = lambda v: np.concatenate(v) if v else np.zeros(0)
    return dict(kx=cat(kx), ky=cat(ky), intensity=cat(I), offsets=np.array(off, dtype=np.int64))
