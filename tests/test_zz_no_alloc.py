"""tm_match_batch_static (no allocation: scratch in a static device array)
against tm_match_batch, through the C ABI, on two calls in a row, the second
with a smaller input; oversized requests and the Fourier route are rejected
before any launch."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _say(*a):
    print("[case]", *a, flush=True)


def _call(tm, fn, lib, polar, norms, prof, N, opts):
    import torch
    B = polar.shape[0]
    dev = polar.device
    tt = torch.full((B, N), -7, dtype=torch.int32, device=dev)
    ts = torch.full((B, N), -7, dtype=torch.int32, device=dev)
    tq = torch.full((B, N), -7.0, dtype=torch.float32, device=dev)
    r = fn(lib._h, polar.data_ptr(), norms.data_ptr(), prof.data_ptr(), B,
           ctypes.byref(opts) if opts is not None else None, N, tt.data_ptr(), ts.data_ptr(),
           tq.data_ptr(), None, None, torch.cuda.current_stream().cuda_stream)
    assert r == tm.TM_OK, tm.last_error()
    torch.cuda.synchronize()
    return tt.cpu().numpy(), ts.cpu().numpy(), tq.cpu().numpy()


def test_static_scratch_matches_allocating_entry_point(tm):
    import torch
    cfg = synth.WORKLOADS[1]
    lib_np = synth.make_library(cfg)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"],
                     synth.px_per_inv_A(cfg), grid)
    N = cfg.N
    for call, (lo, hi, keep, prec) in enumerate([(0, 64, 0.3, tm.TM_PREC_BF16),
                                                 (100, 117, 0.2, tm.TM_PREC_FP8)]):
        _say("static scratch call", call, "patterns", lo, hi, "keep", keep, "prec", prec)
        imgs = synth.make_patterns(cfg, lib_np, range(lo, hi))
        x = torch.from_numpy(imgs).cuda()
        polar, norms, prof = tm.polar_transform(x, grid)
        for opts in (None, tm._Opts(prefilter_keep=keep, prefilter_prec=prec)):
            ref = _call(tm, tm._lib.tm_match_batch, lib, polar, norms, prof, N, opts)
            got = _call(tm, tm._lib.tm_match_batch_static, lib, polar, norms, prof, N, opts)
            for a, b in zip(ref, got):
                assert np.array_equal(a, b)
            assert np.all(got[0] >= 0) and np.all(got[0] < lib.n_total)
    lib.free()


def test_static_scratch_rejects_oversized_and_fourier(tm):
    import torch
    cfg = synth.WORKLOADS[1]
    lib_np = synth.make_library(cfg)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"],
                     synth.px_per_inv_A(cfg), grid, fft=True)
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    L = tm._lib
    _say("static scratch: oversized pre-filter request")
    # 300 base templates, keep 0.3: 90 kept (+ mirrors) and 300 scores per
    # pattern, 1920 bytes; 40000 patterns exceed the 64 MiB array
    o = tm._Opts(prefilter_keep=0.3, prefilter_prec=tm.TM_PREC_BF16)
    r = L.tm_match_batch_static(lib._h, p, p, p, 40000, ctypes.byref(o), 5, p, p, p, None, None,
                                None)
    assert r == tm.TM_EINVAL and "static buffer" in tm.last_error()
    _say("static scratch: Fourier route")
    o = tm._Opts(coarse=tm.TM_COARSE_FFT)
    r = L.tm_match_batch_static(lib._h, p, p, p, 4, ctypes.byref(o), 5, p, p, p, None, None, None)
    assert r == tm.TM_EUNSUPPORTED and "static buffer" in tm.last_error()
    lib.free()
