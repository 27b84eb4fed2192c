"""Seeded synthetic workloads shaped like the paper's (template libraries and
4D-STEM diffraction patterns).

This module is shared by the tests, the benchmark and the oracle-side checks.
It holds none of the indexing method's arithmetic: no polar resampling, no
correlation, no ranking. It only produces inputs:

* template libraries in the paper's template format (Section 2.1): per
  orientation a list of Bragg spots (kx, ky) in 1/Angstrom with intensities,
  stored as CSR arrays (kx, ky, intensity, offsets);
* stacks of diffraction patterns rendered from randomly chosen templates at
  random in-plane angles, with a bright direct beam, background and noise
  (Section 3, Section 4.1 and Section 4.2 give the pattern sizes and detector depth).

Every random draw comes from ``numpy.random.default_rng(SeedSequence([2111,
7347, config_id, stream, index]))`` so any single pattern can be regenerated
on its own (stream 0 = library, 1 = ground truth, 2 = log-normal spot
factors, 3 = detector noise, 4 = arrival/routing of scan rows).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Config", "WORKLOADS", "wavelength_A", "make_library", "make_patterns",
    "ground_truth", "rng_for", "px_per_inv_A", "template_euler", "laue_of",
]

# --------------------------------------------------------------------------
# Physical constants (CODATA 2018) and the electron wavelength.
# --------------------------------------------------------------------------
_H = 6.62607015e-34
_M0 = 9.1093837015e-31
_E = 1.602176634e-19
_C = 299792458.0


def wavelength_A(kv: float) -> float:
    """Relativistic electron wavelength in Angstrom for an accelerating
    voltage in kV (200 kV is the paper's microscope, Section 3)."""
    v = kv * 1e3
    p = math.sqrt(2.0 * _M0 * _E * v * (1.0 + _E * v / (2.0 * _M0 * _C * _C)))
    return _H / p * 1e10


# --------------------------------------------------------------------------
# Workload configurations.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Phase:
    lattice: str            # "fcc", "ortho" or "hcp"
    params: tuple           # (a,) | (a, b, c) | (a, c)
    n_templates: int
    max_spots: int
    sector: str             # "m-3m", "mmm", "6/mmm"
    sampling: str = "spiral"  # "spiral" or "random"


@dataclass(frozen=True)
class Config:
    cid: int
    name: str
    B: int
    H: int
    W: int
    R: int
    n_theta: int
    phases: tuple
    N: int
    dtype: str              # "f32" or "u16"
    lognormal: bool
    kv: float = 200.0
    g_max: float = 1.2      # 1/Angstrom, spots kept within this radius
    s_max: float = 0.05     # linear relrod half-width, 1/Angstrom
    sigma_px: float = 1.5
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def n_templates(self) -> int:
        return sum(p.n_templates for p in self.phases)

    @property
    def cx(self) -> float:
        return self.W / 2.0

    @property
    def cy(self) -> float:
        return self.H / 2.0


FCC_AL = ("fcc", (4.05,))
ORTHO = ("ortho", (5.1, 7.3, 4.6))
HCP = ("hcp", (2.95, 2.95 * 1.59))

WORKLOADS = {
    1: Config(1, "tiny: 64 f32 patterns 128x128, 300 FCC templates <=30 spots",
              B=64, H=128, W=128, R=64, n_theta=360,
              phases=(Phase(*FCC_AL, 300, 30, "m-3m", "random"),), N=5,
              dtype="f32", lognormal=False),
    2: Config(2, "paper-scale: 16384 f32 patterns 256x256, 2000 FCC templates <=100 spots",
              B=16384, H=256, W=256, R=128, n_theta=360,
              phases=(Phase(*FCC_AL, 2000, 100, "m-3m"),), N=5,
              dtype="f32", lognormal=True),
    3: Config(3, "precision form: 16384 f32 patterns 256x256, 20000 orthorhombic templates <=120 spots",
              B=16384, H=256, W=256, R=128, n_theta=360,
              phases=(Phase(*ORTHO, 20000, 120, "mmm"),), N=5,
              dtype="f32", lognormal=True),
    # serving: three resident libraries, rows of 256 uint16 Poisson patterns
    4: Config(4, "serving: rows of 256 u16 patterns 256x256; libraries 2000/8000/20000",
              B=256, H=256, W=256, R=128, n_theta=360,
              phases=(Phase(*FCC_AL, 2000, 100, "m-3m"),), N=5,
              dtype="u16", lognormal=True),
    5: Config(5, "large multi-phase: 262144 u16 patterns 256x256, 50000 templates <=150 spots",
              B=262144, H=256, W=256, R=128, n_theta=360,
              phases=(Phase(*FCC_AL, 5000, 150, "m-3m"),
                      Phase(*HCP, 15000, 150, "6/mmm"),
                      Phase(*ORTHO, 30000, 150, "mmm")), N=10,
              dtype="u16", lognormal=True),
}

# the three resident serving libraries: the 2000 FCC library (same as the
# paper-scale case), an 8000 HCP library and the 20000 orthorhombic library
SERVING_LIBRARIES = {
    0: (Phase(*FCC_AL, 2000, 100, "m-3m"),),
    1: (Phase(*HCP, 8000, 120, "6/mmm"),),
    2: (Phase(*ORTHO, 20000, 120, "mmm"),),
}


def px_per_inv_A(cfg: Config) -> float:
    """Detector calibration: spots at g_max land 4 px inside the polar grid."""
    return (cfg.R - 4) / cfg.g_max


def rng_for(cid: int, stream: int, index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2111, 7347, cid, stream, index]))


# --------------------------------------------------------------------------
# Crystal lattices (reciprocal basis and kinematic structure factor with unit
# atomic scattering factors, Section 2.1).
# --------------------------------------------------------------------------
def _reciprocal_basis(lattice: str, params: tuple) -> np.ndarray:
    """Rows are reciprocal basis vectors b1, b2, b3 (1/Angstrom, no 2*pi)."""
    if lattice == "fcc":
        a = params[0]
        A = np.diag([a, a, a])
    elif lattice == "ortho":
        a, b, c = params
        A = np.diag([a, b, c])
    elif lattice == "hcp":
        a, c = params
        A = np.array([[a, 0.0, 0.0],
                      [-0.5 * a, math.sqrt(3.0) / 2.0 * a, 0.0],
                      [0.0, 0.0, c]])
    else:
        raise ValueError(lattice)
    return np.linalg.inv(A).T


def _atoms(lattice: str) -> np.ndarray:
    if lattice == "fcc":
        return np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    if lattice == "ortho":
        return np.array([[0.0, 0.0, 0.0]])
    if lattice == "hcp":
        return np.array([[0, 0, 0], [1.0 / 3.0, 2.0 / 3.0, 0.5]])
    raise ValueError(lattice)


def _reflections(lattice: str, params: tuple, g_lim: float):
    """All hkl (except 000) with |g| <= g_lim and non-zero structure factor.
    Returns (hkl int array [n,3], g crystal-frame [n,3], |F|^2 [n])."""
    Bm = _reciprocal_basis(lattice, params)
    # bound on |h|,|k|,|l|: |g| >= |component along dual direction|
    # |h_i| = |g . a_i| <= g_lim * |a_i|, with a_i the real-space basis
    A = np.linalg.inv(Bm).T
    lims = [int(math.ceil(g_lim * np.linalg.norm(A[i]))) + 1 for i in range(3)]
    rng = [np.arange(-m, m + 1) for m in lims]
    hkl = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    hkl = hkl[np.any(hkl != 0, axis=1)]
    g = hkl @ Bm
    keep = np.linalg.norm(g, axis=1) <= g_lim
    hkl, g = hkl[keep], g[keep]
    phase = 2.0 * np.pi * (hkl @ _atoms(lattice).T)
    F = np.exp(1j * phase).sum(axis=1)
    F2 = (F * np.conj(F)).real
    keep = F2 > 1e-6
    # stable order by (h, k, l) for tie breaking
    hkl, g, F2 = hkl[keep], g[keep], F2[keep]
    order = np.lexsort((hkl[:, 2], hkl[:, 1], hkl[:, 0]))
    return hkl[order], g[order], F2[order]


# --------------------------------------------------------------------------
# Beam directions on S^2, reduced to a fundamental sector (A03/A04).
# --------------------------------------------------------------------------
def _in_sector(v: np.ndarray, sector: str) -> np.ndarray:
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    if sector == "m-3m":
        return (z >= x) & (x >= y) & (y >= 0)
    if sector == "mmm":
        return (x >= 0) & (y >= 0) & (z >= 0)
    if sector == "6/mmm":
        az = np.arctan2(y, x)
        return (z >= 0) & (az >= 0) & (az <= np.pi / 6 + 1e-15)
    raise ValueError(sector)


def _fold(v: np.ndarray, sector: str) -> np.ndarray:
    """Fold arbitrary unit vectors into the sector (used for random sampling)."""
    if sector == "m-3m":
        a = np.sort(np.abs(v), axis=1)           # ascending: y <= x <= z
        return np.stack([a[:, 1], a[:, 0], a[:, 2]], axis=1)
    if sector == "mmm":
        return np.abs(v)
    if sector == "6/mmm":
        z = np.abs(v[:, 2])
        az = np.mod(np.arctan2(v[:, 1], v[:, 0]), np.pi / 3)
        az = np.where(az > np.pi / 6, np.pi / 3 - az, az)
        rho = np.hypot(v[:, 0], v[:, 1])
        return np.stack([rho * np.cos(az), rho * np.sin(az), z], axis=1)
    raise ValueError(sector)


def _spiral_directions(target: int, sector: str) -> np.ndarray:
    n = max(64, target * 8)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    while True:
        i = np.arange(n, dtype=np.float64)
        z = 1.0 - (2.0 * i + 1.0) / n
        r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        phi = i * golden
        v = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
        v = v[_in_sector(v, sector)]
        if len(v) >= target:
            return v[:target]
        n = int(n * 1.5)


def _directions(phase: Phase, cid: int, phase_idx: int) -> np.ndarray:
    if phase.sampling == "random":
        rng = rng_for(cid, 0, 1000 + phase_idx)
        v = rng.standard_normal((phase.n_templates, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return _fold(v, phase.sector)
    return _spiral_directions(phase.n_templates, phase.sector)


def _bunge_sample_from_crystal(v: np.ndarray) -> np.ndarray:
    """Rotation matrices M (crystal -> sample) with phi1 = 0 such that the
    beam direction v (crystal frame) maps to +z of the sample frame.
    Phi = arccos(v_z), phi2 = atan2(v_x, v_y) (Bunge convention)."""
    Phi = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi2 = np.arctan2(v[:, 0], v[:, 1])
    c, s = np.cos(Phi), np.sin(Phi)
    c2, s2 = np.cos(phi2), np.sin(phi2)
    G = np.zeros((len(v), 3, 3))
    # G: sample -> crystal (rows are crystal coordinates of sample axes^T)
    G[:, 0, 0] = c2
    G[:, 0, 1] = s2 * c
    G[:, 0, 2] = s2 * s
    G[:, 1, 0] = -s2
    G[:, 1, 1] = c2 * c
    G[:, 1, 2] = c2 * s
    G[:, 2, 0] = 0.0
    G[:, 2, 1] = -s
    G[:, 2, 2] = c
    return np.transpose(G, (0, 2, 1))


def _simulate_phase(phase: Phase, cfg: Config, phase_idx: int):
    """Kinematic templates for one phase (Section 2.1): rotate the reciprocal
    lattice by (0, Phi, phi2), excitation error to the Ewald sphere, linear
    relrod shape factor, I = |F|^2 * shape, flat projection onto kx-ky."""
    lam = wavelength_A(cfg.kv)
    k = 1.0 / lam
    hkl, g_c, F2 = _reflections(phase.lattice, phase.params, cfg.g_max + 0.2)
    dirs = _directions(phase, cfg.cid, phase_idx)
    M = _bunge_sample_from_crystal(dirs)
    kx_l, ky_l, I_l, cnt = [], [], [], []
    chunk = 512
    for c0 in range(0, len(dirs), chunk):
        Mc = M[c0:c0 + chunk]
        gs = np.einsum("tij,nj->tni", Mc, g_c)           # [t, n, 3] sample frame
        # incident wave vector along -z: k0 = (0, 0, -1/lambda)
        kk = np.sqrt(gs[..., 0] ** 2 + gs[..., 1] ** 2 + (gs[..., 2] - k) ** 2)
        s_err = k - kk
        shape = np.maximum(0.0, 1.0 - np.abs(s_err) / cfg.s_max)
        I = F2[None, :] * shape
        gxy = np.hypot(gs[..., 0], gs[..., 1])
        ok = (gxy <= cfg.g_max) & (shape > 0.0)
        I = np.where(ok, I, 0.0)
        for t in range(len(Mc)):
            sel = np.nonzero(I[t] > 0.0)[0]
            if len(sel):
                It = I[t, sel]
                sel = sel[It >= 1e-3 * It.max()]
            It = I[t, sel]
            # sort by intensity descending, ties by (h, k, l) (sel is hkl-sorted)
            order = np.argsort(-It, kind="stable")
            sel = sel[order][: phase.max_spots]
            It = I[t, sel]
            if len(It):
                It = It / It.max()
            kx_l.append(gs[t, sel, 0])
            ky_l.append(gs[t, sel, 1])
            I_l.append(It)
            cnt.append(len(sel))
    return kx_l, ky_l, I_l, cnt


_LIB_CACHE: dict = {}


def template_euler(cfg: Config | int, phases: tuple | None = None) -> np.ndarray:
    """(Phi, phi2) in radians of every template of make_library(cfg, phases),
    the Bunge angles of its beam direction with phi1 = 0 (the orientation the
    template was simulated for), [T, 2] float64."""
    if isinstance(cfg, int):
        cfg = WORKLOADS[cfg]
    phases = cfg.phases if phases is None else phases
    out = []
    for pi, phase in enumerate(phases):
        v = _directions(phase, cfg.cid, pi)
        out.append(np.stack([np.arccos(np.clip(v[:, 2], -1.0, 1.0)),
                             np.arctan2(v[:, 0], v[:, 1])], axis=1))
    return np.concatenate(out).astype(np.float64)


def laue_of(phase: Phase) -> str:
    """Laue group of a phase (the symmetry of its sampled sector)."""
    return phase.sector


def make_library(cfg: Config | int, phases: tuple | None = None):
    """CSR template library for a configuration.

    Returns dict(kx, ky, intensity [float64], offsets [int64, T+1],
    phase_of [int32, T]). Templates of all phases are concatenated in phase
    order."""
    if isinstance(cfg, int):
        cfg = WORKLOADS[cfg]
    phases = cfg.phases if phases is None else phases
    key = (cfg.cid, phases, cfg.kv, cfg.g_max, cfg.s_max)
    if key in _LIB_CACHE:
        return _LIB_CACHE[key]
    kx_l, ky_l, I_l, cnt, ph = [], [], [], [], []
    for pi, phase in enumerate(phases):
        a, b, c, n = _simulate_phase(phase, cfg, pi)
        kx_l += a
        ky_l += b
        I_l += c
        cnt += n
        ph += [pi] * len(n)
    offsets = np.zeros(len(cnt) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(cnt)
    lib = dict(
        kx=np.concatenate(kx_l).astype(np.float64) if kx_l else np.zeros(0),
        ky=np.concatenate(ky_l).astype(np.float64) if ky_l else np.zeros(0),
        intensity=np.concatenate(I_l).astype(np.float64) if I_l else np.zeros(0),
        offsets=offsets,
        phase_of=np.asarray(ph, dtype=np.int32),
    )
    _LIB_CACHE[key] = lib
    return lib


# --------------------------------------------------------------------------
# Diffraction patterns.
# --------------------------------------------------------------------------
def ground_truth(cfg: Config, index: int, n_templates: int):
    """(template, mirrored, phi) drawn for one scan point."""
    rng = rng_for(cfg.cid, 1, index)
    t = int(rng.integers(0, n_templates))
    mirrored = bool(rng.integers(0, 2))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))
    return t, mirrored, phi


def _render_spots(img: np.ndarray, xs, ys, amps, sigma: float):
    H, W = img.shape
    off = np.arange(-6, 7)
    rad2 = (4.0 * sigma) ** 2
    x0 = np.rint(xs).astype(np.int64)
    y0 = np.rint(ys).astype(np.int64)
    X = x0[:, None, None] + off[None, None, :]
    Y = y0[:, None, None] + off[None, :, None]
    d2 = (X - xs[:, None, None]) ** 2 + (Y - ys[:, None, None]) ** 2
    val = amps[:, None, None] * np.exp(-d2 / (2.0 * sigma * sigma))
    ok = (d2 <= rad2) & (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
    idx = (Y * W + X)[ok]
    img += np.bincount(idx, weights=val[ok], minlength=H * W).reshape(H, W)


def render_pattern(cfg: Config, lib: dict, index: int, truth=None):
    """Noise-free spot image S (float64) of one scan point, and the truth."""
    T = len(lib["offsets"]) - 1
    t, mirrored, phi = ground_truth(cfg, index, T) if truth is None else truth
    a, b = lib["offsets"][t], lib["offsets"][t + 1]
    kx = lib["kx"][a:b]
    ky = lib["ky"][a:b] * (-1.0 if mirrored else 1.0)
    I = lib["intensity"][a:b]
    if cfg.lognormal and len(I):
        z = rng_for(cfg.cid, 2, index).standard_normal(len(I))
        I = I * np.exp(0.5 * z - 0.125)
    scale = px_per_inv_A(cfg)
    c, s = math.cos(phi), math.sin(phi)
    xs = cfg.cx + scale * (c * kx - s * ky)
    ys = cfg.cy + scale * (s * kx + c * ky)
    S = np.zeros((cfg.H, cfg.W), dtype=np.float64)
    if len(I):
        _render_spots(S, xs, ys, I, cfg.sigma_px)
    amp_db = 4.0 * (I.max() if len(I) else 1.0)
    _render_spots(S, np.array([cfg.cx]), np.array([cfg.cy]), np.array([amp_db]), cfg.sigma_px)
    return S, (t, mirrored, phi), (xs, ys)


def make_pattern(cfg: Config, lib: dict, index: int, truth=None) -> np.ndarray:
    S, _, (xs, ys) = render_pattern(cfg, lib, index, truth)
    rng = rng_for(cfg.cid, 3, index)
    if cfg.dtype == "f32":
        noise = rng.standard_normal((cfg.H, cfg.W), dtype=np.float32)
        return (S + 0.01 + 0.02 * noise).astype(np.float32)
    # Poisson counts: alpha so the mean rate within 2 sigma of the diffracted
    # spot centres is 50 electrons per pixel, plus 0.5 background
    H, W = cfg.H, cfg.W
    yy, xx = np.mgrid[0:H, 0:W]
    near = np.zeros((H, W), dtype=bool)
    r2 = (2.0 * cfg.sigma_px) ** 2
    for x, y in zip(xs, ys):
        xi, yi = int(round(x)), int(round(y))
        y_lo, y_hi = max(0, yi - 4), min(H, yi + 5)
        x_lo, x_hi = max(0, xi - 4), min(W, xi + 5)
        if y_lo >= y_hi or x_lo >= x_hi:
            continue
        sub = (xx[y_lo:y_hi, x_lo:x_hi] - x) ** 2 + (yy[y_lo:y_hi, x_lo:x_hi] - y) ** 2 <= r2
        near[y_lo:y_hi, x_lo:x_hi] |= sub
    mean_s = S[near].mean() if near.any() else 1.0
    alpha = 49.5 / max(mean_s, 1e-12)
    lam = alpha * S + 0.5
    counts = rng.poisson(lam)
    return np.clip(counts, 0, 65535).astype(np.uint16)


def make_patterns(cfg: Config | int, lib: dict, indices) -> np.ndarray:
    """Stack [n, H, W] of patterns (float32 or uint16) for scan indices."""
    if isinstance(cfg, int):
        cfg = WORKLOADS[cfg]
    indices = list(indices)
    dt = np.float32 if cfg.dtype == "f32" else np.uint16
    out = np.empty((len(indices), cfg.H, cfg.W), dtype=dt)
    for n, i in enumerate(indices):
        out[n] = make_pattern(cfg, lib, i)
    return out


def _worker(args):
    cid, lib, lo, hi = args
    return lo, make_patterns(WORKLOADS[cid], lib, range(lo, hi))


def make_patterns_parallel(cfg: Config | int, lib: dict, n: int, workers: int = 8,
                           out: np.ndarray | None = None) -> np.ndarray:
    """Patterns 0..n-1 generated by a process pool; same bytes as
    make_patterns(cfg, lib, range(n))."""
    import multiprocessing as mp
    if isinstance(cfg, int):
        cfg = WORKLOADS[cfg]
    dt = np.float32 if cfg.dtype == "f32" else np.uint16
    if out is None:
        out = np.empty((n, cfg.H, cfg.W), dtype=dt)
    if workers <= 1 or n < 64:
        out[...] = make_patterns(cfg, lib, range(n))
        return out
    step = 128
    jobs = [(cfg.cid, lib, lo, min(n, lo + step)) for lo in range(0, n, step)]
    with mp.get_context("fork").Pool(workers) as pool:
        for lo, arr in pool.imap_unordered(_worker, jobs):
            out[lo:lo + len(arr)] = arr
    return out


# --------------------------------------------------------------------------
# Serving workload: scan rows of 256 uint16 patterns, each routed to one of
# the resident libraries, arriving at a fixed cadence.
# --------------------------------------------------------------------------
SERVING_ROW = 256
SERVING_INTERVAL_S = SERVING_ROW / 4000.0      # 4000 patterns/s


def serving_config(lib_id: int) -> Config:
    base = WORKLOADS[4]
    return Config(4, f"serving row, library {lib_id}", B=SERVING_ROW, H=base.H, W=base.W,
                  R=base.R, n_theta=base.n_theta, phases=SERVING_LIBRARIES[lib_id], N=base.N,
                  dtype="u16", lognormal=True)


def serving_schedule(n_rows: int):
    """(library id per row, arrival offset in seconds per row)."""
    rng = rng_for(4, 4, 0)
    lib_ids = rng.integers(0, len(SERVING_LIBRARIES), n_rows)
    return lib_ids.astype(np.int64), np.arange(n_rows) * SERVING_INTERVAL_S


def serving_row(row_id: int, lib_id: int, lib: dict | None = None, workers: int = 1) -> np.ndarray:
    """Patterns of one scan row: scan indices row_id*256 .. +255 rendered from
    the row's library."""
    cfg = serving_config(lib_id)
    lib = make_library(cfg) if lib is None else lib
    idx = range(row_id * SERVING_ROW, (row_id + 1) * SERVING_ROW)
    if workers > 1:
        import multiprocessing as mp
        chunks = [list(idx)[i:i + 32] for i in range(0, SERVING_ROW, 32)]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.starmap(make_patterns, [(cfg, lib, c) for c in chunks])
        return np.concatenate(parts)
    return make_patterns(cfg, lib, idx)
