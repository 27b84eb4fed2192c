"""GPU parity of the two-stage indexing tools (Section 4.3, custom indexation
procedures): the mask built from the average pattern equals the oracle's
bit for bit, masked polar images match the oracle, and indexing masked
patterns with a second library (unit intensities, a subtracted constant)
matches the oracle's top-N. Runs only on an MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
from conftest import small_library
from parity import PatternRef, check_topn

pytestmark = pytest.mark.gpu

H = W = 128
R, NT = 60, 360
PX = (R - 4) / 1.2


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _render(lib, t, phi, amp, yy, xx):
    a, b = lib["offsets"][t], lib["offsets"][t + 1]
    c, s = np.cos(phi), np.sin(phi)
    img = np.zeros((H, W))
    for kx, ky, w in zip(lib["kx"][a:b], lib["ky"][a:b], lib["intensity"][a:b]):
        x = W / 2 + PX * (c * kx - s * ky)
        y = H / 2 + PX * (s * kx + c * ky)
        img += amp * w * np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * 1.5 ** 2))
    return img


def _two_phase(seed=5, B=12):
    """Every pattern: the same bright matrix pattern; on top, a weak
    precipitate template at a random in-plane angle, and noise."""
    rng = np.random.default_rng(seed)
    matrix = small_library(1, seed + 1, max_spots=12, g_min=0.2)
    prec = small_library(40, seed + 2, max_spots=18, g_min=0.1)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    base = _render(matrix, 0, 0.3, 20.0, yy, xx)
    imgs = np.zeros((B, H, W), dtype=np.float32)
    for b in range(B):
        t = int(rng.integers(0, 40))
        imgs[b] = (base + _render(prec, t, rng.uniform(0, 2 * np.pi), 2.0, yy, xx)
                   + 0.05 * rng.standard_normal((H, W)))
    return prec, imgs


@pytest.mark.parametrize("dtype", ["f32", "u16"])
def test_mask_from_mean_equals_oracle(tm, dtype):
    import torch
    prec, imgs = _two_phase()
    if dtype == "u16":
        imgs = np.clip(np.rint(imgs * 100), 0, 65535).astype(np.uint16)
        thr = 300.0
        x = torch.from_numpy(imgs.view(np.int16)).cuda()
    else:
        thr = 3.0
        x = torch.from_numpy(imgs).cuda()
    _say("mask from mean", dtype, imgs.shape, "threshold", thr)
    m = tm.mask_from_mean(x, thr, n_open=1, n_grow=2).cpu().numpy()
    ref = oracle.matrix_mask64(imgs, thr, n_open=1, n_grow=2)
    assert np.array_equal(m, ref.astype(np.float32))
    assert 0 < (m == 0).sum() < m.size // 4


def test_masked_polar_and_two_stage_index(tm):
    import torch
    prec, imgs = _two_phase()
    _say("two-stage: masked polar and precipitate index", imgs.shape)
    x = torch.from_numpy(imgs).cuda()
    m = tm.mask_from_mean(x, 3.0, n_open=1, n_grow=2)
    mask = m.cpu().numpy().astype(np.float64)
    c = 0.1 * float(imgs.max())
    grid = tm.PolarGrid(R=R, n_theta=NT, cx=W / 2, cy=H / 2)
    lib = tm.Library(prec["kx"], prec["ky"], prec["intensity"], prec["offsets"], PX, grid,
                     unit_intensity=True)
    polar, norms, _ = tm.polar_transform(x, grid, subtract=c, mask=m)
    cpolar, cnorms, _ = tm.polar_transform(x, grid, subtract=c, mask=m, lib=lib)
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, 4))
    ct, cs, cq = (o.cpu().numpy() for o in tm.match_batch(lib, cpolar, cnorms, 4))
    assert np.array_equal(tt, ct) and np.array_equal(ts, cs) and np.array_equal(tq, cq)
    polar = polar.cpu().numpy()
    olib = oracle.OracleLibrary.build(prec, PX, R, NT, unit=True)
    for b in range(len(imgs)):
        P = oracle.polar64(imgs[b], R, NT, subtract=c, mask=mask)
        scale = max(1.0, float(np.abs(imgs[b]).max()))
        assert np.allclose(polar[b], P, rtol=2e-6, atol=2e-6 * scale)
        check_topn(PatternRef(P, olib), tt[b], ts[b], tq[b], margin=1e-4)
