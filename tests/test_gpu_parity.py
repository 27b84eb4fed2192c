"""GPU parity: libtm's HIP path against the FP64 oracle on seeded inputs.

Runs only on an MI355X (marked gpu). Every case prints its name, seed and
shape before touching the GPU."""
import numpy as np
import pytest

import oracle
import synth
from conftest import small_library
from parity import PatternRef, check_topn, scores_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _say(*a):
    print("[case]", *a, flush=True)


def _grid_for(tm, cfg):
    return tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)


def _olib(lib, cfg, **kw):
    return oracle.OracleLibrary.build(lib, synth.px_per_inv_A(cfg), cfg.R, cfg.n_theta, **kw)


def _run(tm, lib_np, imgs, grid, px_per, N, gamma=1.0, subtract=0.0, with_best=False,
         mirror=True, unit=False, grouping=True):
    import torch
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px_per,
                     grid, mirror=mirror, unit_intensity=unit, grouping=grouping)
    _say("layout", lib.layout())
    x = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    polar, norms, prof = tm.polar_transform(x, grid, gamma, subtract)
    out = tm.match_batch(lib, polar, norms, N, with_best=with_best)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in out]
    return lib, polar.cpu().numpy(), norms.cpu().numpy(), prof.cpu().numpy(), res


# --------------------------------------------------------------------------- polar
def _polar_close(got, ref, img):
    scale = max(1.0, float(np.abs(img).max()))
    assert np.allclose(got, ref, rtol=2e-6, atol=2e-6 * scale), float(np.abs(got - ref).max())


def test_polar_c1(tm, c1, c1_lib):
    _say("polar c1 B=64 128x128 R=64")
    import torch
    imgs = synth.make_patterns(c1, c1_lib, range(64))
    grid = _grid_for(tm, c1)
    polar, norms, prof = tm.polar_transform(torch.from_numpy(imgs).cuda(), grid)
    polar, norms, prof = polar.cpu().numpy(), norms.cpu().numpy(), prof.cpu().numpy()
    for b in range(64):
        P = oracle.polar64(imgs[b], c1.R, c1.n_theta)
        _polar_close(polar[b], P, imgs[b])
        assert abs(norms[b] - oracle.norm64(P)) <= 1e-6 * oracle.norm64(P)
        pr = oracle.profile64(P)
        assert np.allclose(prof[:, b], pr, rtol=1e-5, atol=1e-5 * np.abs(pr).max())


@pytest.mark.parametrize("case", ["gamma_sub", "nearest", "offcentre_pad", "u16", "r0dr", "ragged"])
def test_polar_options(tm, case):
    import torch
    rng = np.random.default_rng(sum(map(ord, case)))
    H, W, R, nt = 70, 90, 40, 180
    kw = dict(gamma=1.0, subtract=0.0)
    gk = dict(R=R, n_theta=nt, cx=45.0, cy=35.0)
    imgs = rng.random((3, H, W)).astype(np.float32) * 5.0
    if case == "gamma_sub":
        imgs -= 1.0   # negative pixels: the clamp matters
        kw = dict(gamma=0.5, subtract=0.3)
    elif case == "nearest":
        gk["interp"] = "nearest"
    elif case == "offcentre_pad":
        gk.update(cx=20.3, cy=61.7, R=60)   # many samples outside the image
    elif case == "u16":
        imgs = rng.integers(0, 60000, (3, H, W)).astype(np.uint16)
    elif case == "r0dr":
        gk.update(r0=2.5, dr=0.75)
    elif case == "ragged":
        imgs = rng.random((1, 33, 47)).astype(np.float32)
        H, W = 33, 47
        gk.update(R=30, n_theta=97, cx=23.2, cy=16.9)
    _say("polar option", case, imgs.shape, gk, kw)
    grid = tm.PolarGrid(**gk)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, prof = tm.polar_transform(x, grid, **kw)
    polar, norms = polar.cpu().numpy(), norms.cpu().numpy()
    interp = gk.get("interp", "bilinear")
    for b in range(len(imgs)):
        P = oracle.polar64(imgs[b].astype(np.float64), gk["R"], gk["n_theta"], gk.get("r0", 0.0),
                           gk.get("dr", 1.0), gk["cx"], gk["cy"], kw["gamma"], kw["subtract"],
                           interp)
        _polar_close(polar[b], P, imgs[b].astype(np.float64))
        assert abs(norms[b] - oracle.norm64(P)) <= 1e-6 * oracle.norm64(P) + 1e-9


@pytest.mark.parametrize("case", ["f32", "u16_gamma", "nearest_offcentre", "mask"])
def test_polar_aligned_boxes_many_patterns(tm, case):
    """Widths divisible by 4 stage the LDS boxes as aligned 4-pixel groups
    (one 16-byte store each). B = 700 patterns (more than one workgroup per
    CU over the launch); sampled patterns equal the oracle, and every pattern
    equals the same pattern transformed alone."""
    import torch
    rng = np.random.default_rng(sum(map(ord, case)) + 7)
    B, H, W, R, nt = 700, 72, 96, 40, 180
    gk = dict(R=R, n_theta=nt, cx=47.5, cy=36.0)
    kw = dict(gamma=1.0, subtract=0.0)
    imgs = (rng.random((B, H, W)) * 5.0).astype(np.float32)
    mask = None
    if case == "u16_gamma":
        imgs = rng.integers(0, 60000, (B, H, W)).astype(np.uint16)
        kw = dict(gamma=0.5, subtract=3.0)
    elif case == "nearest_offcentre":
        gk.update(interp="nearest", cx=20.3, cy=61.7, R=60)
    elif case == "mask":
        mask = (rng.random((H, W)) > 0.3).astype(np.float32)
    _say("polar aligned boxes", case, imgs.shape, gk, kw)
    grid = tm.PolarGrid(**gk)
    x = torch.from_numpy(imgs).cuda()
    m = torch.from_numpy(mask).cuda() if mask is not None else None
    polar, norms, prof = tm.polar_transform(x, grid, mask=m, **kw)
    polar, norms, prof = polar.cpu().numpy(), norms.cpu().numpy(), prof.cpu().numpy()
    interp = gk.get("interp", "bilinear")
    for b in list(range(0, B, 97)) + [B - 1]:
        img = imgs[b].astype(np.float64)
        P = oracle.polar64(img, gk["R"], nt, 0.0, 1.0, gk["cx"], gk["cy"], kw["gamma"],
                           kw["subtract"], interp, mask=mask)
        ref_img = oracle.intensity_transform64(img, kw["gamma"], kw["subtract"])
        _polar_close(polar[b], P, ref_img)
        assert abs(norms[b] - oracle.norm64(P)) <= 1e-6 * oracle.norm64(P) + 1e-9
        pr = oracle.profile64(P)
        assert np.allclose(prof[:, b], pr, rtol=1e-5, atol=1e-5 * max(np.abs(pr).max(), 1e-30))
    for b in (0, 255, 256, 511, 699):
        p1, n1, f1 = tm.polar_transform(x[b:b + 1].contiguous(), grid, mask=m, **kw)
        assert np.array_equal(p1.cpu().numpy()[0], polar[b])
        assert n1.cpu().numpy()[0] == norms[b] and np.array_equal(f1.cpu().numpy()[:, 0], prof[:, b])


# --------------------------------------------------------------------------- match
@pytest.mark.parametrize("grouping", [True, False])
def test_match_c1_full(tm, c1, c1_lib, c1_olib, grouping):
    _say("match c1 full B=64 T'=600 N=5 grouping", grouping)
    imgs = synth.make_patterns(c1, c1_lib, range(64))
    grid = _grid_for(tm, c1)
    lib, polar, norms, _, (tt, ts, tq, bq, bs) = _run(tm, c1_lib, imgs, grid,
                                                       synth.px_per_inv_A(c1), 5, with_best=True,
                                                       grouping=grouping)
    lay = lib.layout()
    assert lay["group"] == (3 if grouping else 1) and lay["n_bands"] == 1 and not lay["narrow"]
    exact_contract = exact_tight = 0
    for b in range(64):
        P = oracle.polar64(imgs[b], c1.R, c1.n_theta)
        ref = PatternRef(P, c1_olib)
        exact_contract += check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=False)
        exact_tight += check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)
        # per-template best scores and angles for every template
        assert scores_close(bq[b], ref.best).all()
        srt = np.sort(ref.Q, axis=1)
        am = srt[:, -1] - srt[:, -2]
        clear = am > 2 * np.maximum(1e-5 * np.abs(ref.best), 1e-7) * 2
        assert np.array_equal(bs[b][clear], ref.arg[clear])
    _say("exact ranks: contract", exact_contract, "tight", exact_tight)
    assert exact_tight >= 64 * 5 * 0.5


def test_topn_standalone_matches_sort(tm):
    import torch
    rng = np.random.default_rng(7)
    for B, T, N in ((3, 1000, 5), (2, 70, 64), (5, 4001, 10), (1, 1, 1), (4, 257, 17)):
        _say("topn", B, T, N)
        q = rng.integers(0, 50, (B, T)).astype(np.float32) / 7.0   # many exact ties
        s = rng.integers(0, 360, (B, T)).astype(np.int16)
        tt, ts, tq = tm.topn(torch.from_numpy(q).cuda(), torch.from_numpy(s).cuda(), N)
        tt, ts, tq = tt.cpu().numpy(), ts.cpu().numpy(), tq.cpu().numpy()
        for b in range(B):
            order = np.lexsort((np.arange(T), -q[b].astype(np.float64)))[:N]
            assert np.array_equal(tt[b], order)
            assert np.array_equal(ts[b], s[b][order])
            assert np.array_equal(tq[b], q[b][order])


def test_match_best_then_topn_equals_fused(tm, c1, c1_lib):
    _say("fused top-N == tm_topn(best arrays), c1")
    import torch
    imgs = synth.make_patterns(c1, c1_lib, range(16))
    grid = _grid_for(tm, c1)
    _, _, _, _, (tt, ts, tq, bq, bs) = _run(tm, c1_lib, imgs, grid, synth.px_per_inv_A(c1), 7,
                                            with_best=True)
    t2, s2, q2 = tm.topn(torch.from_numpy(bq).cuda(), torch.from_numpy(bs).cuda(), 7)
    assert np.array_equal(tt, t2.cpu().numpy()) and np.array_equal(ts, s2.cpu().numpy())
    assert np.array_equal(tq, q2.cpu().numpy())


@pytest.mark.parametrize("n_theta", [64, 90, 180, 361, 720])
def test_match_theta_widths(tm, n_theta):
    R = 40
    lib = small_library(30, seed=n_theta, max_spots=12, g_max=1.1, g_min=0.3)
    px = 33.0
    rng = np.random.default_rng(n_theta)
    imgs = rng.random((5, 96, 96)).astype(np.float32)
    _say("theta width", n_theta, "R", R, imgs.shape)
    grid = tm.PolarGrid(R=R, n_theta=n_theta, cx=48.0, cy=48.0)
    olib = oracle.OracleLibrary.build(lib, px, R, n_theta)
    _, _, _, _, (tt, ts, tq, bq, bs) = _run(tm, lib, imgs, grid, px, 6, with_best=True)
    for b in range(5):
        P = oracle.polar64(imgs[b], R, n_theta, cx=48.0, cy=48.0)
        ref = PatternRef(P, olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)
        assert scores_close(bq[b], ref.best).all()


@pytest.mark.parametrize("n_theta,grouping", [(360, True), (360, False), (720, True),
                                              (720, False)])
def test_match_multiband_synthetic(tm, n_theta, grouping):
    """Spots spread over most of 128 rows: the rows do not fit LDS at once and
    stream through it in bands (narrow rows for 360 columns, wide rows for
    720), each wave holding several groups' accumulators across bands."""
    R = 128
    lib = small_library(300, seed=99, max_spots=40, g_max=1.2, g_min=0.05)
    px = (R - 4) / 1.2
    rng = np.random.default_rng(100)
    imgs = rng.random((6, 256, 256)).astype(np.float32)
    _say("multi-band synthetic T=300 R=128 n_theta", n_theta, "grouping", grouping, imgs.shape)
    grid = tm.PolarGrid(R=R, n_theta=n_theta, cx=128.0, cy=128.0)
    olib = oracle.OracleLibrary.build(lib, px, R, n_theta)
    tml, _, _, _, (tt, ts, tq, bq, bs) = _run(tm, lib, imgs, grid, px, 8, with_best=True,
                                              grouping=grouping)
    lay = tml.layout()
    assert lay["n_bands"] > 1 and lay["narrow"] == (n_theta <= 384)
    for b in range(6):
        P = oracle.polar64(imgs[b], R, n_theta)
        ref = PatternRef(P, olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)
        assert scores_close(bq[b], ref.best).all()


@pytest.mark.parametrize("grouping", [True, False])
def test_match_c3_library(tm, grouping):
    """The 20 000-template orthorhombic library (93 touched rows, one band of
    narrow rows) on three patterns of the precision-form scan."""
    cfg = synth.WORKLOADS[3]
    lib = synth.make_library(3)
    imgs = synth.make_patterns(cfg, lib, [0, 4096, 16383])
    _say("c3 library, 3 patterns, T'=40000, grouping", grouping)
    grid = _grid_for(tm, cfg)
    olib = _olib(lib, cfg)
    tml, _, _, _, (tt, ts, tq) = _run(tm, lib, imgs, grid, synth.px_per_inv_A(cfg), 5,
                                      grouping=grouping)
    lay = tml.layout()
    assert lay["n_bands"] == 1 and lay["narrow"] and lay["group"] == (3 if grouping else 1)
    for b in range(3):
        P = oracle.polar64(imgs[b], cfg.R, cfg.n_theta)
        ref = PatternRef(P, olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)


def test_batch_independence_and_determinism(tm, c1, c1_lib):
    _say("batch independence c1")
    imgs = synth.make_patterns(c1, c1_lib, range(40))
    grid = _grid_for(tm, c1)
    px = synth.px_per_inv_A(c1)
    _, _, _, _, full = _run(tm, c1_lib, imgs, grid, px, 5)
    _, _, _, _, again = _run(tm, c1_lib, imgs, grid, px, 5)
    for a, b in zip(full, again):
        assert np.array_equal(a, b)
    for i in (0, 17, 39):
        _, _, _, _, one = _run(tm, c1_lib, imgs[i:i + 1], grid, px, 5)
        for a, b in zip(full, one):
            assert np.array_equal(a[i], b[0])
    # permuting the batch permutes the results
    perm = np.random.default_rng(3).permutation(40)
    _, _, _, _, pr = _run(tm, c1_lib, imgs[perm], grid, px, 5)
    for a, b in zip(full, pr):
        assert np.array_equal(a[perm], b)


def test_edge_cases(tm, c1, c1_lib, c1_olib):
    import torch
    grid = _grid_for(tm, c1)
    px = synth.px_per_inv_A(c1)
    # all-zero pattern: every Q is 0, templates ranked by index at angle 0
    _say("edge: zero pattern")
    z = np.zeros((2, c1.H, c1.W), dtype=np.float32)
    _, _, norms, _, (tt, ts, tq) = _run(tm, c1_lib, z, grid, px, 5)
    assert np.all(norms == 0)
    assert np.array_equal(tt, np.tile(np.arange(5), (2, 1))) and np.all(ts == 0) and np.all(tq == 0)
    # N = T' (complete ordering) on a small library
    _say("edge: N = T'")
    lib = small_library(20, seed=5, g_max=1.1, g_min=0.2)
    olib = oracle.OracleLibrary.build(lib, px, c1.R, c1.n_theta)
    imgs = synth.make_patterns(c1, c1_lib, [3])
    _, _, _, _, (tt, ts, tq) = _run(tm, lib, imgs, grid, px, olib.n_total)
    ref = PatternRef(oracle.polar64(imgs[0], c1.R, c1.n_theta), olib)
    check_topn(ref, tt[0], ts[0], tq[0], margin=1e-4, tight=True)
    # templates whose spots all fall outside the grid, or only the direct beam
    _say("edge: empty templates, no mirrors, unit intensities")
    lib2 = dict(kx=np.array([5.0, 0.0, 0.3, 0.1]), ky=np.array([5.0, 0.0, 0.2, -0.4]),
                intensity=np.array([1.0, 1.0, 0.5, 2.0]),
                offsets=np.array([0, 1, 2, 4], dtype=np.int64))
    olib2 = oracle.OracleLibrary.build(lib2, px, c1.R, c1.n_theta, mirror=False, unit=True)
    _, _, _, _, (tt, ts, tq) = _run(tm, lib2, imgs, grid, px, 3, mirror=False, unit=True)
    ref = PatternRef(oracle.polar64(imgs[0], c1.R, c1.n_theta), olib2)
    check_topn(ref, tt[0], ts[0], tq[0], margin=1e-4, tight=True)
    # B = 0 is a no-op
    _say("edge: B = 0")
    tml = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"], px, grid)
    e = torch.empty((0, c1.H, c1.W), dtype=torch.float32, device="cuda")
    polar, norms, prof = tm.polar_transform(e, grid)
    tt, ts, tq = tm.match_batch(tml, polar, norms, 5)
    assert tt.shape == (0, 5)
    # invalid N is rejected before launch
    with pytest.raises(tm.TMError):
        tm.match_batch(tml, polar, norms, tml.n_total + 1)


def test_library_info(tm, c1, c1_lib, c1_olib):
    grid = _grid_for(tm, c1)
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                     synth.px_per_inv_A(c1), grid)
    info = lib.info()
    assert info["n_templates_total"] == c1_olib.n_total
    assert info["n_spots"] == len(c1_olib.J)
    assert info["device_bytes"] > 0


@pytest.mark.parametrize("case", ["c1", "c3", "multiband"])
def test_compact_rows_equal_full(tm, case):
    """tm_polar_transform_rows with the library's row map writes exactly the
    touched rows of the full polar image (bit for bit), the same norms and
    profiles; the match on the compact image (plain, with per-template best
    arrays, and pre-filtered) equals the match on the full image bit for
    bit."""
    import torch
    if case == "multiband":
        R, nt = 128, 360
        lib_np = small_library(300, seed=99, max_spots=40, g_max=1.2, g_min=0.05)
        px = (R - 4) / 1.2
        imgs = np.random.default_rng(100).random((6, 256, 256)).astype(np.float32)
        grid = tm.PolarGrid(R=R, n_theta=nt, cx=128.0, cy=128.0)
    else:
        cfg = synth.WORKLOADS[1 if case == "c1" else 3]
        lib_np = synth.make_library(cfg)
        px = synth.px_per_inv_A(cfg)
        imgs = synth.make_patterns(cfg, lib_np, range(8))
        grid = _grid_for(tm, cfg)
    _say("compact rows", case, imgs.shape)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid)
    n_rows, row_map = lib.rows()
    x = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    polar, norms, prof = tm.polar_transform(x, grid)
    cpolar, cnorms, cprof = tm.polar_transform(x, grid, lib=lib)
    torch.cuda.synchronize()
    assert cpolar.shape == (len(imgs), n_rows, grid.n_theta)
    touched = sorted({int(j) for j in _olib_rows(lib_np, px, grid)})
    assert len(touched) == n_rows
    assert torch.equal(cpolar, polar[:, touched, :])
    assert torch.equal(cnorms, norms) and torch.equal(cprof, prof)
    N = 5
    full = tm.match_batch(lib, polar, norms, N, with_best=True)
    comp = tm.match_batch(lib, cpolar, cnorms, N, with_best=True)
    for u, v in zip(full, comp):
        assert torch.equal(u, v)
    full = tm.match_batch(lib, polar, norms, N, profiles=prof, prefilter_keep=0.2,
                          prefilter_prec="bf16")
    comp = tm.match_batch(lib, cpolar, cnorms, N, profiles=cprof, prefilter_keep=0.2,
                          prefilter_prec="bf16")
    for u, v in zip(full, comp):
        assert torch.equal(u, v)


def _olib_rows(lib_np, px, grid):
    olib = oracle.OracleLibrary.build(lib_np, px, grid.R, grid.n_theta)
    return np.unique(olib.J)


# --------------------------------------------------------------------------- non-finite input
def test_nonfinite_pattern_is_flagged_and_nan_options_rejected(tm, c1, c1_lib):
    """A pattern holding a NaN or an infinity inside the polar footprint gets
    template -1, angle -1, score NaN on every path (plain, per-template,
    pre-filtered, Fourier route); the other patterns of the batch are
    unaffected. NaN option fractions are rejected before any launch."""
    import ctypes

    import torch
    _say("non-finite patterns c1 B=6")
    imgs = synth.make_patterns(c1, c1_lib, range(6))
    imgs[1, 64, 70] = np.nan
    imgs[4, 60, 64] = np.inf
    grid = _grid_for(tm, c1)
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                     synth.px_per_inv_A(c1), grid, fft=True)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, prof = tm.polar_transform(x, grid)
    bad = [1, 4]
    good = [0, 2, 3, 5]
    ref = tm.match_batch(lib, polar[good].contiguous(), norms[good].contiguous(), 5)
    ref = [r.cpu().numpy() for r in ref]
    runs = {
        "plain": dict(),
        "best": dict(with_best=True),
        "prefilter": dict(profiles=prof, prefilter_keep=1.0, prefilter_prec="bf16"),
        "fourier": dict(coarse="fft"),
    }
    for name, kw in runs.items():
        _say("non-finite path", name)
        out = tm.match_batch(lib, polar, norms, 5, **kw)
        torch.cuda.synchronize()
        tt, ts, tq = (o.cpu().numpy() for o in out[:3])
        assert np.all(tt[bad] == -1) and np.all(ts[bad] == -1) and np.all(np.isnan(tq[bad])), name
        # the other patterns: same best score; same best template and angle
        # where the runner-up is clearly behind (other paths may sum in
        # another order)
        assert np.allclose(tq[good, 0], ref[2][:, 0], rtol=1e-5, atol=1e-7), name
        clear = (ref[2][:, 0] - ref[2][:, 1]) > 1e-4
        assert np.array_equal(tt[good, 0][clear], ref[0][clear, 0]), name
        assert np.array_equal(ts[good, 0][clear], ref[1][clear, 0]), name
        if name == "best":
            bq, bs = out[3].cpu().numpy(), out[4].cpu().numpy()
            assert np.all(np.isnan(bq[bad])) and np.all(bs[bad] == -1)
            assert np.all(np.isfinite(bq[good]))
    # NaN fractions never reach a kernel
    for field in ("prefilter_keep", "rescore_keep"):
        o = tm._Opts()
        setattr(o, field, float("nan"))
        if field == "rescore_keep":
            o.coarse = tm.TM_COARSE_FFT
        r = tm._lib.tm_match_batch(lib._h, polar.data_ptr(), norms.data_ptr(), prof.data_ptr(), 6,
                                   ctypes.byref(o), 5, ref[0].ctypes.data, ref[0].ctypes.data,
                                   ref[0].ctypes.data, None, None, None)
        assert r == tm.TM_EINVAL, field
        assert "outside [0, 1]" in tm.last_error()
    lib.free()
