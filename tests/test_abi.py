"""The C ABI library loads, exports every symbol include/tm.h declares, and
rejects invalid arguments before touching a device. CPU only (no compute)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tm.h")


@pytest.fixture(scope="module")
def tm():
    import paper_2111_07347_amd as tm
    return tm


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(tm):
    names = declared_functions()
    assert len(names) >= 8
    lib = ctypes.CDLL(tm.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tm.EXPORTED)


def test_header_is_plain_c():
    """The boundary uses plain pointers and sizes: no torch or C++ types."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for bad in ("torch", "std::", "at::", "Tensor", "template<", "namespace"):
        assert bad not in src


def test_version(tm):
    assert tm.version().startswith("tm ")


def _grid(tm, **kw):
    return tm._Grid(kw.get("R", 16), kw.get("n_theta", 360), kw.get("r0", 0.0), kw.get("dr", 1.0),
                    kw.get("cx", 8.0), kw.get("cy", 8.0), kw.get("interp", 1))


def test_load_library_argument_errors(tm):
    L = tm._lib
    g = _grid(tm)
    kx = np.zeros(2)
    off = np.array([0, 2], dtype=np.int64)
    h = ctypes.c_void_p()
    # null out pointer
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 1,
                             10.0, ctypes.byref(g), 1, None, None) == tm.TM_EINVAL
    # no templates
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 0,
                             10.0, ctypes.byref(g), 1, None, ctypes.byref(h)) == tm.TM_EINVAL
    assert "n_templates" in tm.last_error()
    # bad grid
    for bad in (_grid(tm, R=0), _grid(tm, n_theta=10), _grid(tm, n_theta=1000), _grid(tm, dr=0.0)):
        assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data,
                                 1, 10.0, ctypes.byref(bad), 1, None,
                                 ctypes.byref(h)) == tm.TM_EINVAL
    # bad calibration, flags, offsets
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 1,
                             -1.0, ctypes.byref(g), 1, None, ctypes.byref(h)) == tm.TM_EINVAL
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 1,
                             10.0, ctypes.byref(g), 64, None, ctypes.byref(h)) == tm.TM_EINVAL
    # the Fourier route needs an even polar width
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 1,
                             10.0, ctypes.byref(_grid(tm, n_theta=361)), 1 | tm.TM_LIB_FFT, None,
                             ctypes.byref(h)) == tm.TM_EUNSUPPORTED
    assert "even" in tm.last_error()
    bad_off = np.array([0, 3, 2], dtype=np.int64)
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, bad_off.ctypes.data,
                             2, 10.0, ctypes.byref(g), 1, None, ctypes.byref(h)) == tm.TM_EINVAL
    assert h.value is None


def test_polar_and_topn_argument_errors(tm):
    L = tm._lib
    g = _grid(tm)
    buf = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    assert L.tm_polar_transform(buf, 1, -1, 16, 16, ctypes.byref(g), 1.0, 0.0, buf, buf, None,
                                None) == tm.TM_EINVAL
    assert L.tm_polar_transform(buf, 7, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, buf, buf, None,
                                None) == tm.TM_EINVAL
    assert L.tm_polar_transform(buf, 1, 1, 16, 16, ctypes.byref(g), 0.0, 0.0, buf, buf, None,
                                None) == tm.TM_EINVAL
    assert L.tm_polar_transform(buf, 1, 1, 0, 16, ctypes.byref(g), 1.0, 0.0, buf, buf, None,
                                None) == tm.TM_EINVAL
    assert L.tm_polar_transform(None, 1, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, buf, buf, None,
                                None) == tm.TM_EINVAL
    # B = 0 is a no-op that succeeds without a device
    assert L.tm_polar_transform(None, 1, 0, 16, 16, ctypes.byref(g), 1.0, 0.0, None, None, None,
                                None) == tm.TM_OK
    assert L.tm_topn(buf, buf, 1, 10, 11, buf, buf, buf, None) == tm.TM_EINVAL
    assert L.tm_topn(buf, buf, 1, 10, 0, buf, buf, buf, None) == tm.TM_EINVAL
    assert L.tm_topn(buf, buf, 1, 100, 65, buf, buf, buf, None) == tm.TM_EINVAL
    assert L.tm_topn(None, buf, 1, 10, 3, buf, buf, buf, None) == tm.TM_EINVAL
    assert L.tm_topn(None, None, 0, 10, 3, None, None, None, None) == tm.TM_OK
    assert L.tm_match_batch(None, buf, buf, None, 1, None, 1, buf, buf, buf, None, None,
                            None) == tm.TM_EINVAL
    e = ctypes.c_double()
    assert L.tm_fft_error_bound(None, ctypes.byref(e)) == tm.TM_EINVAL
    assert L.tm_fft_scores(None, buf, buf, 1, 0, buf, None, None) == tm.TM_EINVAL
    assert L.tm_library_rows(None, None, None) == tm.TM_EINVAL
    # compact polar rows: n_out_rows within [1, R]; without a map it must be R
    assert L.tm_polar_transform_rows(buf, 1, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, None, buf, 0,
                                     buf, buf, None, None) == tm.TM_EINVAL
    assert L.tm_polar_transform_rows(buf, 1, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, None, buf, 17,
                                     buf, buf, None, None) == tm.TM_EINVAL
    assert L.tm_polar_transform_rows(buf, 1, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, None, None, 8,
                                     buf, buf, None, None) == tm.TM_EINVAL
    # mask builder argument checks
    assert L.tm_mask_from_mean(buf, 1, 0, 16, 16, 1.0, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_mask_from_mean(buf, 1, 4, 16, 16, 1.0, -1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_mask_from_mean(buf, 1, 4, 16, 16, float("nan"), 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_mask_from_mean(None, 1, 4, 16, 16, 1.0, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_free_library(None) == tm.TM_OK
    assert L.tm_library_info(None, None, None, None) == tm.TM_EINVAL
    # orientations: exactly one angle source, valid sizes and flags
    assert L.tm_orientations(buf, 4, 1, 360, buf, buf, buf, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_orientations(buf, 4, 1, 360, buf, None, None, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_orientations(buf, 0, 1, 360, buf, buf, None, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_orientations(buf, 4, 2, 360, buf, buf, None, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_orientations(buf, 4, 1, 360, buf, buf, None, 1, 0, buf, None) == tm.TM_EINVAL
    assert L.tm_orientations(None, 4, 1, 360, buf, buf, None, 1, 1, buf, None) == tm.TM_EINVAL
    assert L.tm_ipf_deviation(buf, 3, buf, 3, 1, 3, buf, None) == tm.TM_EINVAL
    assert L.tm_ipf_deviation(buf, 2, buf, 3, 1, 0, buf, None) == tm.TM_EINVAL
    assert L.tm_ipf_deviation(buf, 3, None, 3, 1, 0, buf, None) == tm.TM_EINVAL
    assert L.tm_ipf_deviation(buf, 3, buf, 3, -1, 0, buf, None) == tm.TM_EINVAL
    # library simulation: host crystal arrays are read during validation
    B = np.eye(3) / 4.05
    X = np.zeros((1, 3))
    f = np.ones(1)
    sim = lambda Bm=B, n=1, g_lim=1.4, T=1, k=40.0, smax=0.05, gmax=1.2, rel=1e-3, S=10, o=buf: \
        L.tm_simulate_library(Bm.ctypes.data if Bm is not None else None, X.ctypes.data,
                              f.ctypes.data, n, g_lim, o, T, k, smax, gmax, rel, S, buf, buf,
                              buf, buf, None)
    assert sim(n=0) == tm.TM_EINVAL
    assert sim(n=33) == tm.TM_EINVAL
    assert sim(S=0) == tm.TM_EINVAL
    assert sim(T=-1) == tm.TM_EINVAL
    assert sim(g_lim=0.0) == tm.TM_EINVAL
    assert sim(smax=float("nan")) == tm.TM_EINVAL
    assert sim(rel=-1.0) == tm.TM_EINVAL
    assert sim(o=None) == tm.TM_EINVAL
    assert sim(Bm=np.zeros((3, 3))) == tm.TM_EINVAL                  # singular basis
    assert sim(Bm=np.eye(3) / 40.0) == tm.TM_EUNSUPPORTED            # box too large
    assert sim(Bm=None) == tm.TM_EINVAL
    # preprocessing options
    po = lambda **k: tm._PreOpts(**{**dict(r_box=8, frac=0.5, sigma_min=1.0, sigma_max=6.0,
                                          sigma_blur=1.0, threshold=0.0), **k})
    pre = lambda o, B=1, H=16, W=16, dt=1, p=buf: L.tm_preprocess(p, dt, B, H, W,
                                                                   ctypes.byref(o), buf, None, None)
    assert L.tm_preprocess(buf, 1, 1, 16, 16, None, buf, None, None) == tm.TM_EINVAL
    assert pre(po(), B=-1) == tm.TM_EINVAL
    assert pre(po(), H=0) == tm.TM_EINVAL
    assert pre(po(), dt=5) == tm.TM_EINVAL
    assert pre(po(sigma_min=6.0, sigma_max=1.0)) == tm.TM_EINVAL
    assert pre(po(sigma_blur=-1.0)) == tm.TM_EINVAL
    assert pre(po(sigma_blur=100.0)) == tm.TM_EINVAL
    assert pre(po(threshold=float("nan"))) == tm.TM_EINVAL
    assert pre(po(), p=None) == tm.TM_EINVAL
    assert pre(po(), B=0, p=None) in (tm.TM_OK, tm.TM_ENODEV)


def _has_gpu():
    import torch
    return torch.cuda.is_available()


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_no_device_returns_enodev(tm):
    L = tm._lib
    g = _grid(tm)
    kx = np.array([0.1, 0.2])
    off = np.array([0, 2], dtype=np.int64)
    h = ctypes.c_void_p()
    assert L.tm_load_library(kx.ctypes.data, kx.ctypes.data, kx.ctypes.data, off.ctypes.data, 1,
                             10.0, ctypes.byref(g), 1, None, ctypes.byref(h)) == tm.TM_ENODEV
    assert "device" in tm.last_error()
    buf = ctypes.c_void_p(16)
    assert L.tm_polar_transform(buf, 1, 1, 16, 16, ctypes.byref(g), 1.0, 0.0, buf, buf, None,
                                None) == tm.TM_ENODEV
    assert L.tm_topn(buf, buf, 1, 10, 3, buf, buf, buf, None) == tm.TM_ENODEV


def test_product_does_not_import_oracle():
    """The product path never routes through the oracle."""
    import subprocess
    import sys
    code = ("import sys, paper_2111_07347_amd; "
            "bad=[m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "assert not bad, bad")
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, check=True)
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2111_07347_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
