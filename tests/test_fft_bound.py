"""The FP16 Fourier-route error bound against an emulation of its arithmetic
(CPU). The emulation rounds exactly where the GPU path rounds (float16
spectra with their power-of-two scalings, float32 accumulation, float16
storage of C(k), float16 cosine / sine tables) and must stay within the bound
at every template and shift, also with float16 subnormals flushed to zero."""
import numpy as np
import pytest

import oracle
from conftest import small_library
from fft_bound import (SCALE_P, SCALE_T, SCALE_W, TINY16, fft16_error_bound,
                       spectrum_scale)


def _f16(x, flush):
    y = np.asarray(x, dtype=np.float64).astype(np.float16)
    if flush:
        y = np.where(np.abs(y.astype(np.float64)) < TINY16, np.float16(0), y)
    return y


def _row_max(olib):
    """Largest number of merged pixels of one template in one polar row."""
    key = olib.tid * olib.R + olib.J
    return int(np.bincount(key).max()) if len(key) else 1


def emulate_fft16(P32, olib, flush=False):
    """Scores Q~[T', n_theta] the way the reduced-precision path forms them."""
    P = P32.astype(np.float64)
    n = olib.n_theta
    F = n // 2 + 1
    pn = np.sqrt((P * P).sum())
    sc = spectrum_scale(_row_max(olib), n)
    Ph = np.fft.rfft(P / pn, axis=1) * 2.0 ** SCALE_P
    c16 = _f16(Ph.real.astype(np.float32), flush).astype(np.float32)
    d16 = _f16(Ph.imag.astype(np.float32), flush).astype(np.float32)
    D = oracle.template_images64(olib, 0, olib.n_total)
    tn = np.where(olib.tnorm > 0, olib.tnorm, 1.0)
    Th = np.fft.rfft(D / tn[:, None, None], axis=2) * 2.0 ** SCALE_T
    a16 = _f16(Th.real, flush).astype(np.float32)
    b16 = _f16(Th.imag, flush).astype(np.float32)
    # C(k) = sum_j conj(T) P in float32
    X = (np.einsum("trk,rk->tk", a16, c16, dtype=np.float32)
         + np.einsum("trk,rk->tk", b16, d16, dtype=np.float32))
    Y = (np.einsum("trk,rk->tk", a16, d16, dtype=np.float32)
         - np.einsum("trk,rk->tk", b16, c16, dtype=np.float32))
    resc = np.float32(2.0 ** (sc - SCALE_T - SCALE_P))
    X16 = _f16(X * resc, flush).astype(np.float32)
    Y16 = _f16(Y * resc, flush).astype(np.float32)
    k = np.arange(F)
    ck = np.where((k == 0) | (2 * k == n), 1.0, 2.0)
    s = np.arange(n)
    ang = 2.0 * np.pi * np.outer(k, s) / n
    Wc = _f16(ck[:, None] * np.cos(ang) * 2.0 ** SCALE_W, flush).astype(np.float32)
    Ws = _f16(-ck[:, None] * np.sin(ang) * 2.0 ** SCALE_W, flush).astype(np.float32)
    Z = X16 @ Wc + Y16 @ Ws                      # float32 accumulation
    out = Z * np.float32(2.0 ** -(SCALE_W + sc) / n)
    out[olib.tnorm == 0] = 0.0
    return out


def _exact(P32, olib):
    return oracle.scores64(P32.astype(np.float64), olib)


CASES = [
    # (R, n_theta, n_templates, max_spots, seed)
    (32, 72, 20, 8, 1),
    (64, 360, 12, 30, 2),
    (48, 180, 16, 60, 3),
]


@pytest.mark.parametrize("flush", [False, True])
@pytest.mark.parametrize("R,n_theta,n,spots,seed", CASES)
def test_bound_holds_random_patterns(R, n_theta, n, spots, seed, flush):
    lib = small_library(n, seed, max_spots=spots, g_min=0.05)
    olib = oracle.OracleLibrary.build(lib, (R - 4) / 1.2, R, n_theta)
    eps = fft16_error_bound(R, n_theta, _row_max(olib), int(np.diff(olib.starts).max()))
    rng = np.random.default_rng(seed)
    worst = 0.0
    for trial in range(3):
        P32 = (rng.random((R, n_theta)) ** (1 + 2 * trial)).astype(np.float32)
        err = np.abs(emulate_fft16(P32, olib, flush) - _exact(P32, olib)).max()
        worst = max(worst, err)
    assert worst <= eps, (worst, eps)
    assert eps < 2.5e-3


@pytest.mark.parametrize("flush", [False, True])
def test_bound_holds_pattern_equal_to_template(flush):
    """Largest spectra: the pattern is a template's own image, Q = 1."""
    R, n_theta = 40, 120
    lib = small_library(10, 7, max_spots=40, g_min=0.05)
    olib = oracle.OracleLibrary.build(lib, (R - 4) / 1.2, R, n_theta)
    eps = fft16_error_bound(R, n_theta, _row_max(olib), int(np.diff(olib.starts).max()))
    D = oracle.template_images64(olib, 0, olib.n_total)
    for t in range(olib.T_base):
        P32 = D[t].astype(np.float32)
        if not P32.any():
            continue
        Qe = _exact(P32, olib)
        assert abs(Qe[t].max() - 1.0) < 1e-6
        err = np.abs(emulate_fft16(P32, olib, flush) - Qe).max()
        assert err <= eps, (t, err, eps)


@pytest.mark.parametrize("flush", [False, True])
def test_bound_holds_with_tiny_weights(flush):
    """Weights over six decades push spectra towards float16's subnormals."""
    R, n_theta = 32, 90
    lib = small_library(12, 9, max_spots=20, g_min=0.05)
    rng = np.random.default_rng(10)
    lib["intensity"] = 10.0 ** rng.uniform(-6, 0, len(lib["intensity"]))
    olib = oracle.OracleLibrary.build(lib, (R - 4) / 1.2, R, n_theta)
    eps = fft16_error_bound(R, n_theta, _row_max(olib), int(np.diff(olib.starts).max()))
    P32 = (rng.random((R, n_theta)) ** 8 * 1e-3).astype(np.float32)
    err = np.abs(emulate_fft16(P32, olib, flush) - _exact(P32, olib)).max()
    assert err <= eps, (err, eps)


def test_bound_is_not_vacuous_and_monotone():
    """The bound sits well below typical score gaps and grows with the
    accumulation lengths."""
    e360 = fft16_error_bound(128, 360, 6, 150)
    assert 1.5e-3 < e360 < 2.5e-3
    assert fft16_error_bound(128, 720, 6, 150) > e360
    assert fft16_error_bound(256, 360, 6, 150) > e360
    assert fft16_error_bound(128, 360, 6, 1000) > e360
