"""Orientation of a match and the angular deviation of Eq. (2), in float64
(oracle).

Test infrastructure only (see the package docstring).

Section 2.1: orientations are Bunge Euler angles (phi1, Phi, phi2); all
templates that share Phi and phi2 are related by an in-plane rotation, so the
library samples only (Phi, phi2) with phi1 = 0 and phi1 is found by the
in-plane search. Section 2.2: mirrored templates are the templates reflected
across y = 0 and stand for further orientations. Section 4.1, Eq. (2): the
angular deviation between two orientation maps is the angle between the
vectors shown in each pixel of their inverse-pole-figure maps.

Readings:
* Bunge's g maps sample coordinates to crystal coordinates,
  g = Z(phi2) X(Phi) Z(phi1) with Z, X the passive (frame) rotations about
  z and x; the template of (Phi, phi2) has phi1 = 0.
* Sample frame: x along the image columns, y along the image rows, z = x cross
  y. A match at shift phi (counter-clockwise, +x toward +y, the convention of
  the in-plane search) rotates the template's sample-frame reciprocal
  vectors by phi about z: crystal -> sample becomes Rz(phi) g^T.
* A mirrored template (spots (kx, -ky)) is read as the orientation rotated by
  pi about the sample x axis before the in-plane rotation: (x, y, z) ->
  (x, -y, -z) keeps the projected spots mirrored and is a proper rotation;
  it equals the reflection up to the sign of the out-of-plane component,
  which the projection (flat Ewald sphere) does not see.
* Euler angles are returned with phi1, phi2 in [0, 2 pi) and Phi in [0, pi];
  at Phi = 0 or pi only phi1 +- phi2 is defined and phi2 = 0 is returned.
* Eq. (2) per sample direction d in (x, y, z): v = g d in crystal
  coordinates (the direction an IPF-d map shows), reduced to the fundamental
  sector of the Laue group (the IPF standard triangle), then
  theta = |arccos(v_A . v_P / (|v_A| |v_P|))|.
* Sectors: m-3m: z >= x >= y >= 0; mmm: x, y, z >= 0; 6/mmm (a along x):
  z >= 0 and azimuth in [0, 30 degrees].
"""
from __future__ import annotations

import itertools

import numpy as np

LAUE_GROUPS = ("m-3m", "mmm", "6/mmm")


def rot_z_passive64(a: float) -> np.ndarray:
    """Frame rotation by a about z: coordinates in the rotated frame."""
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_x_passive64(a: float) -> np.ndarray:
    """Frame rotation by a about x."""
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, s], [0.0, -s, c]])


def rot_z_active64(a: float) -> np.ndarray:
    """Rotation of vectors by a about z, counter-clockwise (+x toward +y)."""
    return rot_z_passive64(a).T


def bunge_matrix64(phi1: float, Phi: float, phi2: float) -> np.ndarray:
    """g (sample -> crystal) of Bunge angles: the three frame rotations
    about z, the new x, the new z, applied in that order (Section 2.1)."""
    return rot_z_passive64(phi2) @ rot_x_passive64(Phi) @ rot_z_passive64(phi1)


def euler_from_matrix64(g: np.ndarray) -> np.ndarray:
    """Bunge angles (phi1, Phi, phi2) of a rotation g (sample -> crystal)."""
    g = np.asarray(g, dtype=np.float64)
    Phi = float(np.arccos(np.clip(g[2, 2], -1.0, 1.0)))
    if np.hypot(g[2, 0], g[2, 1]) > 1e-12:
        phi1 = float(np.arctan2(g[2, 0], -g[2, 1]))
        phi2 = float(np.arctan2(g[0, 2], g[1, 2]))
    else:
        # Phi = 0: g = Z(phi1 + phi2); Phi = pi: g[0:2, 0:2] holds phi1 - phi2
        phi1 = float(np.arctan2(g[0, 1], g[0, 0]))
        phi2 = 0.0
    two_pi = 2.0 * np.pi
    return np.array([phi1 % two_pi, Phi, phi2 % two_pi])


def match_orientation64(Phi: float, phi2: float, phi: float, mirrored: bool) -> np.ndarray:
    """Bunge angles of a pattern indexed by the template (Phi, phi2) (or its
    mirror) at in-plane rotation phi (radians)."""
    M = bunge_matrix64(0.0, Phi, phi2).T          # crystal -> sample of the template
    if mirrored:
        M = rot_x_passive64(np.pi).T @ M          # rotation by pi about sample x
    M = rot_z_active64(phi) @ M                   # in-plane rotation found by the search
    return euler_from_matrix64(M.T)


def symmetry_operators64(laue: str) -> np.ndarray:
    """All operators (3x3, proper and improper) of a Laue group, Cartesian
    crystal frame (6/mmm with a along x)."""
    ops = []
    if laue == "m-3m":
        for perm in itertools.permutations(range(3)):
            for signs in itertools.product((1.0, -1.0), repeat=3):
                m = np.zeros((3, 3))
                for i, j in enumerate(perm):
                    m[i, j] = signs[i]
                ops.append(m)
    elif laue == "mmm":
        for signs in itertools.product((1.0, -1.0), repeat=3):
            ops.append(np.diag(signs))
    elif laue == "6/mmm":
        for k in range(6):
            a = k * np.pi / 3.0
            r = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0, 0, 1.0]])
            m = np.diag([1.0, -1.0, 1.0])            # mirror y -> -y
            for base in (r, r @ m):
                ops.append(base)
                ops.append(-base)                    # with inversion
    else:
        raise ValueError(laue)
    return np.array(ops)


def in_sector64(v: np.ndarray, laue: str, tol: float = 1e-12) -> bool:
    x, y, z = v
    if laue == "m-3m":
        return z >= x - tol and x >= y - tol and y >= -tol
    if laue == "mmm":
        return x >= -tol and y >= -tol and z >= -tol
    if laue == "6/mmm":
        return z >= -tol and y >= -tol and y <= np.tan(np.pi / 6.0) * x + tol
    raise ValueError(laue)


def sector_direction64(v: np.ndarray, laue: str) -> np.ndarray:
    """The image of v under the Laue group that lies in the fundamental
    sector (the vector an inverse pole figure shows)."""
    v = np.asarray(v, dtype=np.float64)
    for op in symmetry_operators64(laue):
        w = op @ v
        if in_sector64(w, laue):
            return w
    raise AssertionError("no symmetry image in the sector")


def ipf_deviation64(euler_a, euler_b, laue: str) -> np.ndarray:
    """Eq. (2) for the IPF-x, IPF-y and IPF-z maps of two orientations:
    [3] angles in radians."""
    ga = bunge_matrix64(*euler_a)
    gb = bunge_matrix64(*euler_b)
    out = np.zeros(3)
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        va = sector_direction64(ga @ e, laue)
        vb = sector_direction64(gb @ e, laue)
        c = np.dot(va, vb) / (np.linalg.norm(va) * np.linalg.norm(vb))
        out[d] = abs(np.arccos(np.clip(c, -1.0, 1.0)))
    return out
