"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
closed forms, brute force on tiny inputs, library routines (scipy, numpy.fft),
invariances and the paper's own numbers. CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from conftest import small_library

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lib(R=32, n_theta=72, n=12, seed=0, mirror=True, unit=False, px_per=30.0):
    lib = small_library(n, seed)
    return lib, oracle.OracleLibrary.build(lib, px_per, R, n_theta, mirror=mirror, unit=unit)


def _dense_template(olib, t):
    D = np.zeros((olib.R, olib.n_theta))
    a, b = olib.starts[t], olib.starts[t + 1]
    D[olib.J[a:b], olib.K[a:b]] = olib.Wt[a:b]
    return D


# ---------------------------------------------------------------- P12 golden
def test_p12_angular_step_from_paper():
    """Section 2.2: the in-plane step is 360 degrees over the polar width;
    a 360-column polar image gives 1 degree (stored fixture)."""
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        facts = json.load(f)
    ex = facts["angular_step"]
    assert 360.0 / ex["polar_width"] == ex["delta_phi1_deg"] == 1.0
    # the oracle's angle grid: column k sits at 2*pi*k/n_theta
    x, y = oracle.polar_coords64(2, ex["polar_width"], 0.0, 1.0, 0.0, 0.0)
    ang = np.degrees(np.arctan2(y[1], x[1]))
    assert abs(ang[1] - ang[0] - ex["delta_phi1_deg"]) < 1e-12
    assert facts["prefilter_keep_fraction"]["value"] == 0.1


def test_electron_wavelength_200kv():
    """200 kV electrons (Section 3): relativistic lambda = 0.025079 A."""
    assert abs(synth.wavelength_A(200.0) - 0.025079) < 5e-7


# ---------------------------------------------------------------- P9 analytic polar
def test_p9_polar_reproduces_bilinear_functions():
    """Bilinear interpolation reproduces f = a + b x + c y + d x y exactly, so
    the polar image of such an image is f at the sample points (pins the
    x = column, y = row, theta from +x to +y conventions)."""
    H, W = 40, 48
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c, d = 0.3, 0.7, -0.45, 0.013
    img = a + b * xx + c * yy + d * xx * yy
    R, n_theta, cx, cy = 15, 90, 23.0, 19.0
    P = oracle.polar64(img, R, n_theta, 0.0, 1.0, cx, cy)
    r = np.arange(R)[:, None]
    th = 2 * np.pi * np.arange(n_theta)[None, :] / n_theta
    X = cx + r * np.cos(th)
    Y = cy + r * np.sin(th)
    assert np.allclose(P, a + b * X + c * Y + d * X * Y, rtol=0, atol=1e-11)


def test_p9_constant_image_and_radial_rows():
    img = np.full((64, 64), 2.5)
    P = oracle.polar64(img, 30, 360)
    assert np.allclose(P, 2.5, rtol=1e-15, atol=0)
    # a radially symmetric image sampled at integer radii along the axes
    yy, xx = np.mgrid[0:64, 0:64].astype(np.float64)
    img = np.hypot(xx - 32, yy - 32)
    P = oracle.polar64(img, 30, 360)
    for k in (0, 90, 180, 270):          # samples fall on pixel centres
        assert np.allclose(P[:, k], np.arange(30), atol=1e-12)


def test_intensity_transform_order():
    """Clamp, gamma, then subtract (Section 2.2 and Section 4.3)."""
    x = np.array([-1.0, 0.0, 0.25, 4.0])
    assert np.allclose(oracle.intensity_transform64(x, 0.5, 0.1), [-0.1, -0.1, 0.4, 1.9])
    assert np.allclose(oracle.intensity_transform64(x, 1.0, 0.0), x)
    assert np.allclose(oracle.intensity_transform64(x, 1.0, 1.0), x - 1.0)


# ---------------------------------------------------------------- P6 library cross-checks
def test_p6_polar_equals_scipy_map_coordinates():
    rng = np.random.default_rng(3)
    img = rng.standard_normal((50, 60))
    R, n_theta, cx, cy = 40, 128, 27.5, 24.0      # reaches outside: zero padding
    P = oracle.polar64(img, R, n_theta, 0.5, 0.9, cx, cy)
    x, y = oracle.polar_coords64(R, n_theta, 0.5, 0.9, cx, cy)
    ref = ndimage.map_coordinates(img, [y.ravel(), x.ravel()], order=1,
                                  mode="grid-constant", cval=0.0).reshape(R, n_theta)
    assert np.allclose(P, ref, rtol=0, atol=1e-12)


def test_p6_numerator_equals_fft_cross_correlation():
    lib, olib = _lib()
    rng = np.random.default_rng(4)
    P = rng.standard_normal((olib.R, olib.n_theta))
    Q = oracle.scores64(P, olib, pnorm=1.0)
    for t in range(olib.n_total):
        D = _dense_template(olib, t)
        cc = np.fft.irfft(np.conj(np.fft.rfft(D, axis=1)) * np.fft.rfft(P, axis=1),
                          n=olib.n_theta, axis=1).sum(axis=0)
        tn = olib.tnorm[t]
        assert np.allclose(Q[t] * tn, cc, atol=1e-10)


def test_p6_prefilter_equals_matmul_and_stable_sort():
    lib, olib = _lib(n=40, seed=5)
    rng = np.random.default_rng(6)
    P = rng.random((olib.R, olib.n_theta))
    profT = oracle.radial_profiles64(olib)
    # profile of a base template: dense template summed along theta
    for t in range(olib.T_base):
        assert np.allclose(profT[t], _dense_template(olib, t).sum(axis=1))
    kept, cos = oracle.prefilter64(P.sum(axis=1), profT, 0.25)
    pP = P.sum(axis=1)
    ref = (profT @ pP) / (np.linalg.norm(profT, axis=1) * np.linalg.norm(pP))
    assert np.allclose(cos, ref)
    order = np.argsort(-ref, kind="stable")[: math.ceil(0.25 * olib.T_base)]
    assert list(kept) == list(order)


# ---------------------------------------------------------------- P1 Cauchy-Schwarz
@pytest.mark.parametrize("roll", [0, 1, 17, 71])
def test_p1_template_image_scores_one(roll):
    lib, olib = _lib()
    for t in range(olib.n_total):
        if olib.tnorm[t] == 0:
            continue
        P = np.roll(_dense_template(olib, t), roll, axis=1)
        Q = oracle.scores64(P, olib)
        assert np.all(np.abs(Q) <= 1.0 + 1e-14)
        assert abs(Q[t, roll] - 1.0) < 1e-14
        best, arg = oracle.match_exact64(P, olib)
        assert abs(best[t] - 1.0) < 1e-14
        # the first maximising shift of template t is the roll unless the
        # template is rotationally symmetric (then an earlier shift also fits)
        D = _dense_template(olib, t)
        assert np.array_equal(np.roll(D, arg[t], axis=1), P)
        assert arg[t] <= roll


# ---------------------------------------------------------------- P2 brute force, Cartesian
def test_p2_cartesian_rotated_template_equals_polar_shift():
    """For every template and shift: rotate the raw spots in Cartesian space
    by s bins, round each rotated spot to its pixel, sample the raw image at
    that pixel's Cartesian position with scipy, sum with the merged weights.
    Must equal the polar-path numerator."""
    R, n_theta, px = 24, 60, 20.0
    lib = small_library(8, seed=11, g_max=1.1)
    olib = oracle.OracleLibrary.build(lib, px, R, n_theta, mirror=False)
    rng = np.random.default_rng(12)
    H = W = 56
    img = rng.random((H, W))
    cx, cy = 28.0, 27.0
    P = oracle.polar64(img, R, n_theta, 0.0, 1.0, cx, cy)
    C = oracle.scores64(P, olib, pnorm=1.0) * olib.tnorm[:, None]
    for t in range(olib.T_base):
        a, b = lib["offsets"][t], lib["offsets"][t + 1]
        kx, ky, w = lib["kx"][a:b], lib["ky"][a:b], lib["intensity"][a:b]
        for s in range(n_theta):
            ang = 2 * np.pi * s / n_theta
            rx = np.cos(ang) * kx - np.sin(ang) * ky
            ry = np.sin(ang) * kx + np.cos(ang) * ky
            rho = px * np.hypot(rx, ry)
            j = np.rint(rho)
            k = np.mod(np.rint(np.arctan2(ry, rx) * n_theta / (2 * np.pi)), n_theta)
            ok = j < R
            # merge by pixel, then sample each pixel's Cartesian position
            pix = {}
            for jj, kk, ww in zip(j[ok], k[ok], w[ok]):
                pix[(int(jj), int(kk))] = pix.get((int(jj), int(kk)), 0.0) + ww
            tot = 0.0
            for (jj, kk), ww in pix.items():
                th = 2 * np.pi * kk / n_theta
                xs, ys = cx + jj * np.cos(th), cy + jj * np.sin(th)
                v = ndimage.map_coordinates(img, [[ys], [xs]], order=1, mode="grid-constant")[0]
                tot += ww * v
            assert abs(tot - C[t, s]) < 1e-10, (t, s)


# ---------------------------------------------------------------- P3 one-bin rotation
def test_p3_roll_by_one_bin():
    lib, olib = _lib(n=20, seed=7)
    rng = np.random.default_rng(8)
    P = rng.random((olib.R, olib.n_theta))
    best, arg = oracle.match_exact64(P, olib)
    best1, arg1 = oracle.match_exact64(np.roll(P, 1, axis=1), olib)
    assert np.allclose(best, best1, rtol=0, atol=1e-15)
    assert np.array_equal(arg1, (arg + 1) % olib.n_theta)


def test_p3_rendered_rotation_by_one_bin(c1, c1_olib):
    """A Cartesian pattern rendered from template t at shift s0 and at s0 + 1
    (Gaussian spots at the template pixels' Cartesian positions) has its
    best angle for t move by exactly one bin."""
    rng = np.random.default_rng(5)
    checked = 0
    for t in rng.choice(c1_olib.n_total, 8, replace=False):
        if c1_olib.tnorm[t] == 0:
            continue
        sub = c1_olib.subset([t])
        s0 = int(rng.integers(0, c1.n_theta))
        got = []
        for s in (s0, s0 + 1):
            img = _render_pixels(c1_olib, t, s, c1.H, c1.W, c1.cx, c1.cy, sigma=1.5)
            P = oracle.polar64(img, c1.R, c1.n_theta)
            got.append(int(np.argmax(oracle.scores64(P, sub)[0])))
        # rotationally symmetric templates resolve to the lowest equivalent shift
        D = _dense_template(c1_olib, t)
        per = next(p for p in range(1, c1.n_theta + 1)
                   if np.array_equal(np.roll(D, p, axis=1), D))
        assert got[0] == s0 % per and got[1] == (s0 + 1) % per
        checked += 1
    assert checked >= 6


# ---------------------------------------------------------------- P4 rendered pattern
def _render_pixels(olib, t, s0, H, W, cx, cy, sigma=1.0):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.zeros((H, W))
    a, b = olib.starts[t], olib.starts[t + 1]
    for j, k, w in zip(olib.J[a:b], olib.K[a:b], olib.Wt[a:b]):
        th = 2 * np.pi * ((k + s0) % olib.n_theta) / olib.n_theta
        x, y = cx + j * np.cos(th), cy + j * np.sin(th)
        img += w * np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * sigma ** 2))
    return img


def test_p4_rendered_template_scores_maximal():
    R, n_theta = 40, 180
    # spots at 16..36 px, where one 2-degree bin spans at least half a pixel
    lib = small_library(16, seed=21, g_max=1.1, g_min=0.5)
    olib = oracle.OracleLibrary.build(lib, 33.0, R, n_theta)
    H = W = 96
    rng = np.random.default_rng(22)
    for t in range(0, olib.n_total, 3):
        if olib.tnorm[t] == 0:
            continue
        s0 = int(rng.integers(0, n_theta))
        img = _render_pixels(olib, t, s0, H, W, 48.0, 48.0)
        tt, ss, qq, _ = oracle.index_pattern64(img, olib, 3, cx=48.0, cy=48.0)
        # expected: template t at s0 unless an identical pixel set (rotated)
        # with a lower template index or a smaller shift exists
        Dt = np.roll(_dense_template(olib, t), s0, axis=1)
        equiv = [(u, s) for u in range(olib.n_total) for s in range(n_theta)
                 if np.array_equal(np.roll(_dense_template(olib, u), s, axis=1), Dt)]
        assert (int(tt[0]), int(ss[0])) == min(equiv)


# ---------------------------------------------------------------- P5 invariance
def test_p5_scale_invariance():
    lib, olib = _lib(n=20, seed=9)
    rng = np.random.default_rng(10)
    img = rng.random((70, 70))
    t1, s1, q1, _ = oracle.index_pattern64(img, olib, 6, cx=35.0, cy=35.0)
    t2, s2, q2, _ = oracle.index_pattern64(7.5 * img, olib, 6, cx=35.0, cy=35.0)
    lib3 = dict(lib, intensity=lib["intensity"] * 3.25)
    olib3 = oracle.OracleLibrary.build(lib3, 30.0, olib.R, olib.n_theta)
    t3, s3, q3, _ = oracle.index_pattern64(img, olib3, 6, cx=35.0, cy=35.0)
    assert np.array_equal(t1, t2) and np.array_equal(s1, s2)
    assert np.array_equal(t1, t3) and np.array_equal(s1, s3)
    assert np.allclose(q1, q2, rtol=1e-13) and np.allclose(q1, q3, rtol=1e-13)


# ---------------------------------------------------------------- P7 brute-force top-N
def test_p7_topn_brute_force():
    R, n_theta = 12, 36
    lib = small_library(9, seed=31, g_max=0.9)
    olib = oracle.OracleLibrary.build(lib, 12.0, R, n_theta)
    rng = np.random.default_rng(32)
    P = rng.integers(0, 4, (R, n_theta)).astype(np.float64)   # integer image: many ties
    pn = math.sqrt(float((P * P).sum()))
    # pure-python triple loop over (template, shift, pixel)
    triples = []
    pix = oracle.template_pixels64(lib["kx"], lib["ky"], lib["intensity"], lib["offsets"],
                                   12.0, R, n_theta)
    for t, (J, K, Wt) in enumerate(pix):
        tn = math.sqrt(sum(w * w for w in Wt))
        for s in range(n_theta):
            num = 0.0
            for j, k, w in zip(J, K, Wt):
                num += w * P[j, (k + s) % n_theta]
            q = num / (pn * tn) if tn > 0 else 0.0
            triples.append((-q, t, s))
    triples.sort()
    seen, expect = set(), []
    for nq, t, s in triples:
        if t not in seen:
            seen.add(t)
            expect.append((t, s, -nq))
    for N in (1, 4, len(pix)):
        best, arg = oracle.match_exact64(P, olib, pn)
        t, s, q = oracle.topn64(best, arg, N)
        assert [(int(a), int(b)) for a, b in zip(t, s)] == [(e[0], e[1]) for e in expect[:N]]
        assert np.allclose(q, [e[2] for e in expect[:N]], atol=1e-14)


# ---------------------------------------------------------------- P8 prefilter special case
def test_p8_prefilter_keep_all_equals_exact():
    lib, olib = _lib(n=25, seed=41)
    rng = np.random.default_rng(42)
    img = rng.random((70, 70))
    t1, s1, q1, _ = oracle.index_pattern64(img, olib, 7, cx=35.0, cy=35.0)
    t2, s2, q2, ids = oracle.index_pattern_prefiltered64(img, olib, 7, keep=1.0, cx=35.0, cy=35.0)
    assert len(ids) == olib.n_total
    assert np.array_equal(t1, t2) and np.array_equal(s1, s2) and np.allclose(q1, q2)


# ---------------------------------------------------------------- P10 equivariance
def test_p10_template_permutation():
    lib, olib = _lib(n=15, seed=51, mirror=False)
    rng = np.random.default_rng(52)
    P = rng.random((olib.R, olib.n_theta))
    best, arg = oracle.match_exact64(P, olib)
    perm = rng.permutation(olib.T_base)
    off = lib["offsets"]
    kx, ky, I, no = [], [], [], [0]
    for t in perm:
        kx.append(lib["kx"][off[t]:off[t + 1]])
        ky.append(lib["ky"][off[t]:off[t + 1]])
        I.append(lib["intensity"][off[t]:off[t + 1]])
        no.append(no[-1] + off[t + 1] - off[t])
    lib2 = dict(kx=np.concatenate(kx), ky=np.concatenate(ky), intensity=np.concatenate(I),
                offsets=np.array(no))
    olib2 = oracle.OracleLibrary.build(lib2, 30.0, olib.R, olib.n_theta, mirror=False)
    best2, arg2 = oracle.match_exact64(P, olib2)
    assert np.allclose(best2, best[perm], atol=1e-15) and np.array_equal(arg2, arg[perm])


# ---------------------------------------------------------------- P11 mirror identity
def test_p11_mirror_identity():
    """Flipping the image about y = cy maps the score of template t at shift
    s onto the score of mirror(t) at -s."""
    lib, olib = _lib(n=10, seed=61)
    rng = np.random.default_rng(62)
    H = W = 64
    cy = 32
    img = rng.random((H, W))
    flip = np.zeros_like(img)
    for y in range(H):
        if 0 <= 2 * cy - y < H:
            flip[y] = img[2 * cy - y]
    P = oracle.polar64(img, olib.R, olib.n_theta, cx=32.0, cy=float(cy))
    Pf = oracle.polar64(flip, olib.R, olib.n_theta, cx=32.0, cy=float(cy))
    Q = oracle.scores64(P, olib)
    Qf = oracle.scores64(Pf, olib)
    T = olib.T_base
    n = olib.n_theta
    neg = (-np.arange(n)) % n
    for t in range(T):
        assert np.allclose(Qf[t], Q[T + t][neg], atol=1e-12)
        assert np.allclose(Qf[T + t], Q[t][neg], atol=1e-12)


def test_mirror_pixels_are_reflected_columns():
    lib, olib = _lib(n=10, seed=71)
    T = olib.T_base
    for t in range(T):
        a, b = olib.starts[t], olib.starts[t + 1]
        c, d = olib.starts[T + t], olib.starts[T + t + 1]
        base = sorted(zip(olib.J[a:b], olib.K[a:b], olib.Wt[a:b]))
        mir = sorted(zip(olib.J[c:d], (-olib.K[c:d]) % olib.n_theta, olib.Wt[c:d]))
        assert [(j, k) for j, k, _ in base] == [(j, k) for j, k, _ in mir]
        assert np.allclose([w for *_, w in base], [w for *_, w in mir])


# ---------------------------------------------------------------- template pixel rules
def test_template_pixels_rounding_merge_and_drop():
    px, R, n = 10.0, 8, 8          # 45 degree bins
    kx = np.array([0.0, 0.31, 0.0, 0.7, 0.701, 0.3 * np.cos(np.pi / 8 + 1e-9), 0.0])
    ky = np.array([0.0, 0.0, 0.52, 0.0, 0.0, 0.3 * np.sin(np.pi / 8 + 1e-9), 0.9])
    w = np.array([5.0, 1.0, 2.0, 0.5, 0.25, 3.0, 9.0])
    J, K, W = oracle.template_pixels64(kx, ky, w, [0, 7], px, R, n, mirror=False)[0]
    got = {(int(j), int(k)): float(x) for j, k, x in zip(J, K, W)}
    # direct beam dropped; rho 3.1 -> j 3; 5.2 at 90 deg -> (5, 2);
    # 7.0 and 7.01 merge at (7, 0); 3.0 at 22.5+ deg -> k = 1; 9.0 -> j 9 >= R dropped
    assert got == {(3, 0): 1.0, (5, 2): 2.0, (7, 0): 0.75, (3, 1): 3.0}
    J2, K2, W2 = oracle.template_pixels64(kx, ky, w, [0, 7], px, R, n, mirror=False,
                                          unit=True, keep_direct_beam=True)[0]
    got2 = {(int(j), int(k)): float(x) for j, k, x in zip(J2, K2, W2)}
    assert got2 == {(0, 0): 1.0, (3, 0): 1.0, (5, 2): 1.0, (7, 0): 2.0, (3, 1): 1.0}


def test_zero_norm_scores_zero():
    lib, olib = _lib(n=5, seed=81)
    P = np.zeros((olib.R, olib.n_theta))
    best, arg = oracle.match_exact64(P, olib)
    assert np.all(best == 0) and np.all(arg == 0)
    t, s, q = oracle.topn64(best, arg, 3)
    assert list(t) == [0, 1, 2] and list(s) == [0, 0, 0]


def test_oracle_does_not_import_product():
    import subprocess
    import sys
    code = ("import sys, oracle, synth; "
            "bad=[m for m in sys.modules if m.startswith('paper_2111_07347_amd')]; "
            "assert not bad, bad")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([sys.executable, "-c", code], cwd=root, check=True)


# ------------------------------------------------ Fourier route along theta
def test_fft_route_numerator_equals_shift_sum_brute_force():
    """Section 2.2: the in-plane search is a circular cross-correlation along
    theta. On a tiny case the Fourier-route numerator must equal the plain
    double sum over (row, column) of T[j, c] * P[j, (c + s) mod n_theta]."""
    lib, olib = _lib(R=12, n_theta=20, n=5, seed=11, px_per=9.0)
    rng = np.random.default_rng(12)
    P = rng.standard_normal((olib.R, olib.n_theta))
    C = oracle.fft_numerators64(P, olib, 0, olib.n_total)
    for t in range(olib.n_total):
        D = _dense_template(olib, t)
        for s in range(olib.n_theta):
            ref = 0.0
            for j in range(olib.R):
                for c in range(olib.n_theta):
                    ref += D[j, c] * P[j, (c + s) % olib.n_theta]
            assert abs(C[t, s] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_fft_route_dense_images_and_mirror_reflection():
    """Dense template images carry exactly the merged weights; the mirror
    image is the base image reflected k -> -k (Section 2.2, Fig. 2 f)."""
    lib, olib = _lib(n=10, seed=13)
    D = oracle.template_images64(olib, 0, olib.n_total)
    T = olib.T_base
    for t in range(olib.n_total):
        assert np.array_equal(D[t], _dense_template(olib, t))
        assert np.isclose(np.sqrt((D[t] ** 2).sum()), olib.tnorm[t], rtol=1e-15)
    refl = np.roll(D[:T, :, ::-1], 1, axis=2)        # column k -> (-k) mod n_theta
    assert np.allclose(D[T:], refl, atol=0)


def test_fft_route_matches_direct_search():
    """The Fourier route reaches the direct search's result: best Q to
    1e-12 and the same smallest maximising shift wherever the best shift is
    unique by more than 1e-9."""
    lib, olib = _lib(n=30, seed=14)
    rng = np.random.default_rng(15)
    for trial in range(3):
        P = rng.random((olib.R, olib.n_theta)) ** 3
        best_d, arg_d = oracle.match_exact64(P, olib)
        best_f, arg_f = oracle.fft_match64(P, olib, chunk=7)
        assert np.allclose(best_f, best_d, rtol=0, atol=1e-12)
        Q = oracle.scores64(P, olib)
        for t in range(olib.n_total):
            q = np.sort(Q[t])[::-1]
            if q[0] - q[1] > 1e-9:
                assert arg_f[t] == arg_d[t]


# ------------------------------------------------- two-stage indexing mask
def test_mask_morphology_equals_scipy():
    """Erosion / dilation with the 3x3 square element and an unset border
    equal scipy.ndimage's binary morphology (library-routine cross-check)."""
    from scipy import ndimage
    rng = np.random.default_rng(21)
    b = rng.random((37, 41)) > 0.45
    st = np.ones((3, 3), dtype=bool)
    for n in (1, 2, 3):
        assert np.array_equal(oracle.binary_erode64(b, n),
                              ndimage.binary_erosion(b, st, iterations=n, border_value=0))
        assert np.array_equal(oracle.binary_dilate64(b, n),
                              ndimage.binary_dilation(b, st, iterations=n, border_value=0))


def test_mask_removes_matrix_reflections_keeps_precipitate_spot():
    """A reflection present in every pattern (matrix) is masked with its
    tails; a spot present in one pattern only (precipitate) survives; a
    single bright noise pixel in the average is removed by the opening."""
    H = W = 48
    yy, xx = np.mgrid[0:H, 0:W]
    matrix = 10.0 * np.exp(-((xx - 12) ** 2 + (yy - 30) ** 2) / (2 * 1.5 ** 2))
    imgs = np.repeat(matrix[None], 8, axis=0)
    imgs[3] += 10.0 * np.exp(-((xx - 36) ** 2 + (yy - 10) ** 2) / (2 * 1.5 ** 2))
    imgs[:, 5, 40] = 50.0                       # one-pixel noise feature in every pattern
    m = oracle.matrix_mask64(imgs, threshold=2.0, n_open=1, n_grow=2)
    assert m[30, 12] == 0.0 and m[30, 15] == 0.0 and m[33, 12] == 0.0   # core and tails
    assert m[10, 36] == 1.0                    # precipitate spot: mean 1.25 < 2
    assert m[5, 40] == 1.0                     # opened away
    assert set(np.unique(m)) <= {0.0, 1.0}


def test_masked_polar_special_cases():
    """Mask of ones = no mask; mask of zeros = zero polar image; a mask
    multiplies the transformed pattern (gamma, then subtraction) before
    resampling."""
    rng = np.random.default_rng(22)
    img = rng.random((40, 44)) * 3.0
    R, nt = 18, 72
    P = oracle.polar64(img, R, nt, gamma=0.5, subtract=0.2)
    assert np.array_equal(oracle.polar64(img, R, nt, gamma=0.5, subtract=0.2,
                                         mask=np.ones_like(img)), P)
    assert not oracle.polar64(img, R, nt, gamma=0.5, subtract=0.2,
                              mask=np.zeros_like(img)).any()
    m = (rng.random(img.shape) > 0.5).astype(float)
    ref = oracle.bilinear64((np.sqrt(img) - 0.2) * m, *oracle.polar_coords64(R, nt, 0.0, 1.0,
                                                                            22.0, 20.0))
    assert np.allclose(oracle.polar64(img, R, nt, gamma=0.5, subtract=0.2, mask=m), ref,
                       rtol=0, atol=1e-14)


# ------------------------------------------------- sub-bin in-plane angle
def _render_polar_spots(olib, t, phi_bins, sigma=1.2):
    """Polar image of template t's pixels as Gaussians along theta at a
    fractional rotation (in bins): an exactly known sub-bin angle."""
    P = np.zeros((olib.R, olib.n_theta))
    a, b = olib.starts[t], olib.starts[t + 1]
    k = np.arange(olib.n_theta)
    for j, kk, w in zip(olib.J[a:b], olib.K[a:b], olib.Wt[a:b]):
        d = (k - (kk + phi_bins) + olib.n_theta / 2) % olib.n_theta - olib.n_theta / 2
        P[j] += w * np.exp(-d ** 2 / (2 * sigma ** 2))
    return P


def test_refined_angle_recovers_fractional_rotation():
    """A template's own (Gaussian-broadened) image rotated by s0 + f bins:
    the best shift is within a bin of s0 + f and the parabola recovers f to
    a few hundredths of a bin (the peak is nearly parabolic)."""
    lib, olib = _lib(R=24, n_theta=180, n=6, seed=31, px_per=10.0)
    for t in range(olib.T_base):
        if olib.starts[t + 1] - olib.starts[t] < 2:
            continue
        for s0, f in ((17, 0.0), (40, 0.3), (111, -0.45)):
            P = _render_polar_spots(olib, t, s0 + f)
            Q = oracle.scores64(P, olib.subset([t]))[0]
            s = int(np.argmax(Q))
            ang = oracle.refine_angle64(P, olib, t, s)
            want = ((s0 + f) * 2.0) % 360.0              # 2 degrees per bin
            assert abs((ang - want + 180) % 360 - 180) < 0.06 * 2.0, (t, s0, f, ang, want)


def test_refined_angle_moves_one_bin_with_a_rolled_image():
    """Rolling the polar image by one column moves the refined angle by
    exactly one bin (the three scores are the same numbers, relabelled)."""
    lib, olib = _lib(n=8, seed=32)
    rng = np.random.default_rng(33)
    P = rng.random((olib.R, olib.n_theta)) ** 4
    best, arg = oracle.match_exact64(P, olib)
    step = 360.0 / olib.n_theta
    for t in range(olib.n_total):
        a0 = oracle.refine_angle64(P, olib, t, int(arg[t]))
        a1 = oracle.refine_angle64(np.roll(P, 1, axis=1), olib, t, (int(arg[t]) + 1) % olib.n_theta)
        assert abs((a1 - a0 - step + 180) % 360 - 180) < 1e-9


# ------------------------------------------------- orientations and Eq. (2)
def _random_euler(rng, n):
    return np.stack([rng.uniform(0, 2 * np.pi, n), np.arccos(rng.uniform(-1, 1, n)),
                     rng.uniform(0, 2 * np.pi, n)], axis=1)


def test_bunge_matrix_equals_scipy_intrinsic_zxz():
    """Bunge g (sample -> crystal) is the transpose of scipy's intrinsic
    z-x'-z'' rotation with the same three angles."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(40)
    for e in _random_euler(rng, 50):
        want = Rotation.from_euler("ZXZ", e).as_matrix().T
        assert np.allclose(oracle.bunge_matrix64(*e), want, atol=1e-13)


def test_euler_round_trip_and_degenerate_axes():
    rng = np.random.default_rng(41)
    for e in _random_euler(rng, 50):
        back = oracle.euler_from_matrix64(oracle.bunge_matrix64(*e))
        d = (back - e + np.pi) % (2 * np.pi) - np.pi
        assert np.allclose(d, 0.0, atol=1e-9), (e, back)
    for Phi in (0.0, np.pi):
        for a, c in ((0.3, 1.1), (5.9, 4.0)):
            g = oracle.bunge_matrix64(a, Phi, c)
            back = oracle.euler_from_matrix64(g)
            assert back[2] == 0.0 and back[1] == Phi
            assert np.allclose(oracle.bunge_matrix64(*back), g, atol=1e-12)


def test_match_orientation_reproduces_rotated_and_mirrored_spots():
    """Section 2.1/2.2: the orientation of a match at in-plane angle phi maps
    the crystal's reciprocal vectors onto the template's spots rotated by phi
    (counter-clockwise, +x toward +y), or onto the mirrored spots (kx, -ky)
    rotated by phi for a mirrored template."""
    rng = np.random.default_rng(42)
    gc = rng.standard_normal((20, 3))                    # crystal-frame g vectors
    for _ in range(20):
        Phi, phi2 = np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi)
        phi = rng.uniform(0, 2 * np.pi)
        tmpl = (oracle.bunge_matrix64(0.0, Phi, phi2).T @ gc.T).T[:, :2]   # template spots
        c, s = np.cos(phi), np.sin(phi)
        for mirrored in (False, True):
            sp = tmpl * np.array([1.0, -1.0]) if mirrored else tmpl
            want = np.stack([c * sp[:, 0] - s * sp[:, 1], s * sp[:, 0] + c * sp[:, 1]], axis=1)
            e = oracle.match_orientation64(Phi, phi2, phi, mirrored)
            got = (oracle.bunge_matrix64(*e).T @ gc.T).T[:, :2]
            assert np.allclose(got, want, atol=1e-12), (mirrored, e)
            assert 0 <= e[0] < 2 * np.pi and 0 <= e[1] <= np.pi and 0 <= e[2] < 2 * np.pi


@pytest.mark.parametrize("laue, order", [("m-3m", 48), ("mmm", 8), ("6/mmm", 24)])
def test_laue_group_is_a_group_and_sector_is_fundamental(laue, order):
    ops = oracle.symmetry_operators64(laue)
    assert len(ops) == order
    keys = {tuple(np.round(o, 9).ravel()) for o in ops}
    assert len(keys) == order
    for a in ops[:8]:
        for b in ops:
            assert tuple(np.round(a @ b, 9).ravel()) in keys       # closed under products
    rng = np.random.default_rng(43)
    for v in rng.standard_normal((200, 3)):
        w = oracle.sector_direction64(v, laue)
        assert oracle.in_sector64(w, laue)
        assert np.isclose(np.linalg.norm(w), np.linalg.norm(v))
        assert any(np.allclose(w, o @ v, atol=1e-12) for o in ops)
        # exactly one image lies strictly inside the sector for a generic v
        inside = sum(all(np.isclose(o @ v, w, atol=1e-12)) for o in ops)
        assert inside == 1
    if laue == "m-3m":
        for v in rng.standard_normal((50, 3)):
            a = np.sort(np.abs(v))
            assert np.allclose(oracle.sector_direction64(v, laue), [a[1], a[0], a[2]])


def test_eq2_closed_forms():
    """Eq. (2): identical and symmetry-equivalent orientations deviate by 0;
    a rotation about the beam leaves IPF-z unchanged; beam along [001] vs
    [101] and [111] (cubic) gives 45 degrees and arccos(1/sqrt(3))."""
    rng = np.random.default_rng(44)
    for laue in ("m-3m", "mmm", "6/mmm"):
        ops = oracle.symmetry_operators64(laue)
        proper = [o for o in ops if np.linalg.det(o) > 0]
        for e in _random_euler(rng, 10):
            assert np.allclose(oracle.ipf_deviation64(e, e, laue), 0.0, atol=1e-7)
            S = proper[rng.integers(len(proper))]
            e2 = oracle.euler_from_matrix64(S @ oracle.bunge_matrix64(*e))
            assert np.allclose(oracle.ipf_deviation64(e, e2, laue), 0.0, atol=1e-6)
            e3 = e.copy()
            e3[0] = (e3[0] + 0.3) % (2 * np.pi)      # phi1 rotates about the sample z axis
            assert oracle.ipf_deviation64(e, e3, laue)[2] < 1e-7
    # beam (sample z) along crystal [001]: Phi = 0; along [101]: Phi = 45 deg,
    # phi2 = 90 deg (v = (sin phi2 sin Phi, cos phi2 sin Phi, cos Phi))
    z001 = np.array([0.0, 0.0, 0.0])
    z101 = np.array([0.0, np.pi / 4, np.pi / 2])
    z111 = np.array([0.0, np.arccos(1 / np.sqrt(3)), np.pi / 4])
    assert np.isclose(oracle.ipf_deviation64(z001, z101, "m-3m")[2], np.pi / 4, atol=1e-12)
    assert np.isclose(oracle.ipf_deviation64(z001, z111, "m-3m")[2],
                      np.arccos(1 / np.sqrt(3)), atol=1e-12)
    assert np.isclose(oracle.ipf_deviation64(z101, z111, "m-3m")[2],
                      np.arccos(2 / np.sqrt(6)), atol=1e-12)


# ------------------------------------------------ library simulation (2.1)
FCC_A = 4.05
K_200KV = 1.0 / synth.wavelength_A(200.0)
FCC_ATOMS = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=float)


def test_reciprocal_grid_equals_brute_force():
    from oracle import simulate as osim
    Bm = np.diag([1 / 5.1, 1 / 7.3, 1 / 4.6])
    hkl, g = osim.reciprocal_grid64(Bm, 1.0)
    want = [(h, k, l) for h in range(-12, 13) for k in range(-12, 13) for l in range(-12, 13)
            if (h, k, l) != (0, 0, 0) and (h / 5.1) ** 2 + (k / 7.3) ** 2 + (l / 4.6) ** 2 <= 1.0]
    assert [tuple(r) for r in hkl] == sorted(want)
    assert np.allclose(g, hkl * np.array([1 / 5.1, 1 / 7.3, 1 / 4.6]))


def test_structure_factors_textbook():
    """FCC: F F* = 16 for unmixed hkl, 0 for mixed. HCP (atoms at 0 and
    (1/3, 2/3, 1/2)): 4, 0, 1, 3 by (h + 2k mod 3, l parity)."""
    from oracle import simulate as osim
    rng = np.random.default_rng(60)
    hkl = rng.integers(-6, 7, (300, 3))
    F2 = osim.structure_factor_sq64(hkl, FCC_ATOMS, np.ones(4))
    unmixed = np.all(hkl % 2 == 0, axis=1) | np.all(hkl % 2 == 1, axis=1)
    assert np.allclose(F2, np.where(unmixed, 16.0, 0.0), atol=1e-9)
    F2 = osim.structure_factor_sq64(hkl, [[0, 0, 0], [1 / 3, 2 / 3, 0.5]], np.ones(2))
    r3 = (hkl[:, 0] + 2 * hkl[:, 1]) % 3
    lo = hkl[:, 2] % 2 == 1
    want = np.where(r3 == 0, np.where(lo, 0.0, 4.0), np.where(lo, 3.0, 1.0))
    assert np.allclose(F2, want, atol=1e-9)


def test_excitation_error_ewald_geometry():
    """Points on the sphere through the origin with centre (0, 0, k) have
    s = 0, points inside s > 0; near the origin s = gz - gxy^2 / (2k) to
    second order."""
    from oracle import simulate as osim
    rng = np.random.default_rng(61)
    u = rng.standard_normal((50, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    on = np.array([0, 0, K_200KV]) + K_200KV * u
    assert np.allclose(osim.excitation_error64(on, K_200KV), 0.0, atol=1e-10)
    assert np.all(osim.excitation_error64(np.array([0, 0, K_200KV]) + 0.5 * K_200KV * u, K_200KV) > 0)
    g = rng.uniform(-1.0, 1.0, (50, 3)) * np.array([1, 1, 0.05])
    approx = g[:, 2] - (g[:, 0] ** 2 + g[:, 1] ** 2) / (2 * K_200KV)
    err = np.abs(osim.excitation_error64(g, K_200KV) - approx)
    assert np.all(err < 5 * np.linalg.norm(g, axis=1) ** 3 / K_200KV ** 2 + 1e-12)


def _fcc_zone(Phi, phi2, max_spots=200):
    from oracle import simulate as osim
    _, g, F2 = osim.reflections64(np.eye(3) / FCC_A, FCC_ATOMS, np.ones(4), 1.4)
    return osim.simulate_template64(g, F2, Phi, phi2, K_200KV, 0.05, 1.2, 1e-3, max_spots)


def test_fcc_001_zone_axis_pattern():
    """Beam along [001]: the zero-order Laue zone only (l = 0), h and k both
    even, on a square grid of spacing 2/a within g_max; brightest nearest
    the centre (the Ewald sphere leaves the plane as g^2 / 2k); equal
    intensities in lexicographic (h, k) order."""
    kx, ky, I = _fcc_zone(0.0, 0.0)
    want = sorted([(h, k) for h in range(-8, 9, 2) for k in range(-8, 9, 2)
                   if (h, k) != (0, 0) and np.hypot(h, k) / FCC_A <= 1.2],
                  key=lambda hk: (hk[0] ** 2 + hk[1] ** 2, hk))
    got = np.stack([kx, ky], axis=1) * FCC_A
    assert np.allclose(got, np.array(want, dtype=float), atol=1e-9)
    # zero layer: |s| = k - sqrt(k^2 + g^2) exactly = g^2 / (k + sqrt(k^2 + g^2))
    g2 = kx ** 2 + ky ** 2
    s = g2 / (K_200KV + np.sqrt(K_200KV ** 2 + g2))
    assert np.all(np.diff(I) <= 1e-15) and np.isclose(I[0], 1.0)
    assert np.allclose(I, (1 - s / 0.05) / (1 - s[0] / 0.05), atol=1e-12)


def test_phi2_rotates_a_zone_pattern_in_plane():
    """With Phi = 0 the orientation is a rotation about the beam: phi2
    rotates the projected spots counter-clockwise by phi2."""
    kx0, ky0, I0 = _fcc_zone(0.0, 0.0)
    a = 0.7
    kx, ky, I = _fcc_zone(0.0, a)
    rot = np.stack([np.cos(a) * kx0 - np.sin(a) * ky0, np.sin(a) * kx0 + np.cos(a) * ky0], 1)
    got = np.stack([kx, ky], axis=1)
    key = lambda p: tuple(np.round(p, 9))
    assert sorted(map(key, got)) == sorted(map(key, rot))
    assert np.allclose(np.sort(I), np.sort(I0))


def test_simulation_equals_workload_generator_library():
    """The oracle's simulation reproduces the workload generator's own
    kinematical library (an independent implementation) for the tiny case."""
    from oracle import simulate as osim
    cfg = synth.WORKLOADS[1]
    lib = synth.make_library(cfg)
    o = osim.simulate_library64(np.eye(3) / FCC_A, FCC_ATOMS, np.ones(4), cfg.g_max + 0.2,
                                synth.template_euler(cfg), 1 / synth.wavelength_A(cfg.kv),
                                cfg.s_max, cfg.g_max, 1e-3, cfg.phases[0].max_spots)
    assert np.array_equal(o["offsets"], lib["offsets"])
    for key in ("kx", "ky", "intensity"):
        assert np.allclose(o[key], lib[key], atol=1e-12)


# ------------------------------------------------ preprocessing (Section 4.1)
@pytest.mark.parametrize("sigma", [0.7, 1.0, 2.5, 6.0])
def test_gaussian_equals_scipy_reflect(sigma):
    rng = np.random.default_rng(80)
    img = rng.random((37, 50))
    want = ndimage.gaussian_filter(img, sigma, mode="reflect", truncate=4.0)
    assert np.allclose(oracle.gaussian64(img, sigma), want, atol=1e-12)
    # an image narrower than the kernel folds the mirror more than once
    small = rng.random((5, 7))
    assert np.allclose(oracle.gaussian64(small, sigma),
                       ndimage.gaussian_filter(small, sigma, mode="reflect", truncate=4.0),
                       atol=1e-12)


def test_dog_of_constant_is_zero_and_linear():
    rng = np.random.default_rng(81)
    img = rng.random((40, 40))
    d = lambda a: oracle.gaussian64(a, 1.0) - oracle.gaussian64(a, 6.0)
    assert np.allclose(d(np.full((40, 40), 3.5)), 0.0, atol=1e-12)
    assert np.allclose(d(img + 7.0), d(img), atol=1e-12)


def test_beam_centre_brute_force_and_symmetric_spots():
    img = np.zeros((32, 32))
    img[16, 16] = img[16, 17] = 5.0                 # two equal pixels: the midpoint
    assert oracle.beam_centre64(img, 4, 0.5) == (16.5, 16.0)
    yy, xx = np.mgrid[0:64, 0:64].astype(float)
    for x0, y0 in ((31.0, 33.0), (34.5, 29.5)):     # pixel- and half-pixel-centred spots
        spot = np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / (2 * 1.7 ** 2))
        cx, cy = oracle.beam_centre64(spot, 8, 0.3)
        assert abs(cx - x0) < 1e-12 and abs(cy - y0) < 1e-12
    # brute force on a random box: centroid of the kept pixels
    rng = np.random.default_rng(82)
    img = rng.random((20, 24))
    H, W = img.shape
    pts = [(x, y, img[y, x]) for y in range(H) for x in range(W)
           if abs(x - W / 2) <= 3 and abs(y - H / 2) <= 3]
    m = max(v for _, _, v in pts)
    keep = [(x, y, v) for x, y, v in pts if v >= 0.6 * m]
    s = sum(v for _, _, v in keep)
    want = (sum(x * v for x, _, v in keep) / s, sum(y * v for _, y, v in keep) / s)
    assert np.allclose(oracle.beam_centre64(img, 3, 0.6), want, atol=1e-13)
    assert oracle.beam_centre64(np.zeros((8, 8)), 2, 0.5) == (4.0, 4.0)


def test_shift_integer_fraction_and_round_trip():
    rng = np.random.default_rng(83)
    img = rng.random((16, 20))
    s = oracle.shift_image64(img, 3.0, -2.0)        # out(x, y) = in(x + 3, y - 2)
    want = np.zeros_like(img)
    want[2:, :-3] = img[:-2, 3:]
    assert np.allclose(s, want, atol=1e-14)
    s = oracle.shift_image64(img, 0.25, 0.0)
    assert np.allclose(s[:, :-1], 0.75 * img[:, :-1] + 0.25 * img[:, 1:], atol=1e-14)
    # a bilinear function is reproduced exactly away from the border
    yy, xx = np.mgrid[0:16, 0:20].astype(float)
    f = 1.0 + 0.3 * xx - 0.2 * yy + 0.01 * xx * yy
    s = oracle.shift_image64(f, 1.3, -0.6)
    g = 1.0 + 0.3 * (xx + 1.3) - 0.2 * (yy - 0.6) + 0.01 * (xx + 1.3) * (yy - 0.6)
    assert np.allclose(s[2:-2, 1:-3], g[2:-2, 1:-3], atol=1e-12)


def test_preprocess_centres_an_offset_beam():
    """A pattern whose direct beam sits 3.4 px right and 2.25 px down of the
    centre: after preprocessing the beam's centroid is back at (W/2, H/2)."""
    H = W = 64
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    img = 10 * np.exp(-((xx - 35.4) ** 2 + (yy - 34.25) ** 2) / (2 * 1.5 ** 2)) + 0.2
    out, (cx, cy) = oracle.preprocess64(img, r_box=8, frac=0.05, sigma_min=0.0,
                                        sigma_max=0.0, sigma_blur=0.0)
    # a thresholded centroid of an off-grid spot is biased by a small part of
    # a pixel (less the lower the threshold)
    assert abs(cx - 35.4) < 0.03 and abs(cy - 34.25) < 0.03
    c2 = oracle.beam_centre64(out, 8, 0.05)
    assert abs(c2[0] - 32.0) < 0.03 and abs(c2[1] - 32.0) < 0.03


# ---------------------------------------------------------------- nearest-pixel sampling
def _asymmetric_image(H=31, W=37, seed=71):
    """Distinct values everywhere (no symmetry can hide a swapped axis)."""
    rng = np.random.default_rng(seed)
    return rng.permutation(H * W).reshape(H, W).astype(np.float64) + 1.0


def test_nearest_on_pixel_centres_fixes_axes():
    """Integer radii along the four axes put the sample points on pixel
    centres: polar column 0 walks along +x (image columns), column n/4 along
    +y (image rows), and each sample returns exactly that pixel."""
    img = _asymmetric_image()
    cx, cy, R, n = 17.0, 14.0, 12, 360
    P = oracle.polar64(img, R, n, 0.0, 1.0, cx, cy, interp="nearest")
    j = np.arange(R)
    assert np.array_equal(P[:, 0], img[14, 17 + j])
    assert np.array_equal(P[:, 90], img[14 + j, 17])
    assert np.array_equal(P[:, 180], img[14, 17 - j])
    assert np.array_equal(P[:, 270], img[14 - j, 17])


def test_nearest_equals_brute_force_closest_centre():
    """Away from ties, the nearest sample is the pixel whose centre is
    closest in Euclidean distance, searched over a lattice extended past the
    border (a closest centre outside the image gives 0)."""
    img = _asymmetric_image(23, 29, seed=72)
    H, W = img.shape
    R, n, cx, cy = 18, 97, 13.3, 10.6
    P = oracle.polar64(img, R, n, 0.35, 0.93, cx, cy, interp="nearest")
    x, y = oracle.polar_coords64(R, n, 0.35, 0.93, cx, cy)
    ys, xs = np.mgrid[-3:H + 3, -3:W + 3]
    for jj in range(R):
        for kk in range(n):
            d2 = (xs - x[jj, kk]) ** 2 + (ys - y[jj, kk]) ** 2
            flat = np.sort(d2.ravel())
            assert flat[1] - flat[0] > 1e-9          # no tie at this sample
            i = np.argmin(d2)
            yi, xi = ys.ravel()[i], xs.ravel()[i]
            inside = 0 <= yi < H and 0 <= xi < W
            want = img[yi, xi] if inside else 0.0
            assert P[jj, kk] == want, (jj, kk)


def test_nearest_half_pixel_ties_round_half_to_even():
    """Reading: exact half-pixel coordinates round half to even (IEEE
    default), so x = 10.5 -> 10, 11.5 -> 12, 12.5 -> 12, 13.5 -> 14."""
    img = _asymmetric_image()
    P = oracle.polar64(img, 4, 360, 0.5, 1.0, 10.0, 6.0, interp="nearest")
    assert list(P[:, 0]) == [img[6, c] for c in (10, 12, 12, 14)]
    # along +y: y = 6.5, 7.5, 8.5, 9.5 -> rows 6, 8, 8, 10
    assert list(P[:, 90]) == [img[r, 10] for r in (6, 8, 8, 10)]


def test_nearest_outside_image_is_zero():
    img = _asymmetric_image(20, 20, seed=73)
    P = oracle.polar64(img, 40, 360, 0.0, 1.0, 10.0, 10.0, interp="nearest")
    x, y = oracle.polar_coords64(40, 360, 0.0, 1.0, 10.0, 10.0)
    out = (np.rint(x) < 0) | (np.rint(x) > 19) | (np.rint(y) < 0) | (np.rint(y) > 19)
    assert out.any() and np.all(P[out] == 0.0)
    assert np.all(P[~out] != 0.0)


# ---------------------------------------------------------------- pre-filter ranking
def _distinct_profile_library(T=18, seed=81, dup=(3, 11)):
    """Base templates of 3-6 spots on distinct rows with random weights
    (pairwise non-proportional radial profiles), except that template dup[1]
    repeats the spots of dup[0] exactly."""
    rng = np.random.default_rng(seed)
    kx, ky, w, off = [], [], [], [0]
    spots = []
    for t in range(T):
        n = int(rng.integers(3, 7))
        rad = rng.choice(np.arange(6, 28), size=n, replace=False) / 30.0 + 1e-3
        ang = rng.uniform(0, 2 * np.pi, n)
        spots.append((rad * np.cos(ang), rad * np.sin(ang), rng.uniform(0.2, 1.0, n)))
    spots[dup[1]] = spots[dup[0]]
    for x, y, i in spots:
        kx += list(x)
        ky += list(y)
        w += list(i)
        off.append(off[-1] + len(x))
    lib = dict(kx=np.array(kx), ky=np.array(ky), intensity=np.array(w),
               offsets=np.array(off, dtype=np.int64))
    return oracle.OracleLibrary.build(lib, 30.0, 32, 72)


def test_prefilter_own_image_has_cosine_one_and_ranks_first():
    """A polar image equal to template t's pixel image, at any roll, has the
    same radial profile as t, so the cosine is 1 (Cauchy-Schwarz equality)
    and t is kept first; an exact duplicate of t ties and the lower index
    comes first."""
    olib = _distinct_profile_library()
    profT = oracle.radial_profiles64(olib)
    u = profT / np.linalg.norm(profT, axis=1, keepdims=True)
    C = u @ u.T
    np.fill_diagonal(C, 0.0)
    C[3, 11] = C[11, 3] = 0.0
    assert C.max() < 1 - 1e-6                      # no other proportional pair
    for t in range(olib.T_base):
        for roll in (0, 5, 41):
            P = np.roll(_dense_template(olib, t), roll, axis=1)
            prof = oracle.profile64(P)
            assert prof.shape == (olib.R,)
            kept, cos = oracle.prefilter64(prof, profT, 0.2)
            assert abs(cos[t] - 1.0) < 1e-12
            first = 3 if t in (3, 11) else t
            assert kept[0] == first
            if t in (3, 11):
                assert kept[1] == 11 and cos[3] == cos[11]
            assert np.all(cos <= 1.0 + 1e-12)


def test_prefilter_cosine_equals_half_squared_distance_of_unit_profiles():
    """For unit vectors u, v: u . v = 1 - |u - v|^2 / 2, a formula that
    involves no dot product; checks that both profiles are normalised."""
    olib = _distinct_profile_library(seed=82)
    profT = oracle.radial_profiles64(olib)
    rng = np.random.default_rng(83)
    pP = rng.random(olib.R) * 3.0
    _, cos = oracle.prefilter64(pP, profT, 0.5)
    u = profT / np.sqrt((profT ** 2).sum(axis=1, keepdims=True))
    v = pP / np.sqrt((pP ** 2).sum())
    assert np.allclose(cos, 1.0 - ((u - v) ** 2).sum(axis=1) / 2.0, rtol=0, atol=1e-12)


def test_prefilter_invariances_and_count():
    """The ranking does not change when the polar image is rolled along
    theta or scaled, or when every weight of one template is scaled; the
    kept count is ceil(f T) (reading: 'a tenth' of 25 keeps 3)."""
    olib = _distinct_profile_library(T=25, seed=84, dup=(0, 0))
    profT = oracle.radial_profiles64(olib)
    rng = np.random.default_rng(85)
    P = rng.random((olib.R, olib.n_theta))
    k0, c0 = oracle.prefilter64(oracle.profile64(P), profT, 0.1)
    assert len(k0) == 3
    k1, c1 = oracle.prefilter64(oracle.profile64(np.roll(P, 13, axis=1)), profT, 0.1)
    k2, c2 = oracle.prefilter64(oracle.profile64(7.5 * P), profT, 0.1)
    pT = profT.copy()
    pT[int(k0[1])] *= 40.0
    k3, c3 = oracle.prefilter64(oracle.profile64(P), pT, 0.1)
    for k, c in ((k1, c1), (k2, c2), (k3, c3)):
        assert list(k) == list(k0)
        assert np.allclose(c, c0, rtol=0, atol=1e-13)
