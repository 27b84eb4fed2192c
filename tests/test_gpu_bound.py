"""GPU: the window upper bounds of every template's best score
(tm_bound_scores) and the exact search built on them (tm_match_batch with
coarse = TM_COARSE_BOUND), which must return the plain path's top-N.

The bound's definition: with M[j, x] = max(0, max_{0 <= d < wlen} P[j, x + d])
(win = ceil(n_theta / 4), wlen = min(win + dl, n_theta), dl = 4 win - n_theta,
columns mod n_theta) the largest of the 4 window sums
sum_i w_i M[j_i, k_i + S win - e_iS] / ||P|| bounds max_s Q(t, s), where
e_iS = dl when floor(k_i / win) + S >= 4 and 0 otherwise (the kernel
reads the 4 maxima of a pixel from columns k_i mod win + q win, q = 0..3;
0 whenever 4 divides n_theta). The tests
check that every bound is at least the plain path's float32 best score of
its template, and that it is that window sum (computed here in float64 from
the same polar image) up to the documented float16 rounding up and float32
margins. Runs only on an MI355X (marked gpu)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from conftest import small_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _say(*a):
    print("[case]", *a, flush=True)


def _setup(tm, cfg, lib_np, idx, **polar_kw):
    import torch
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"],
                     synth.px_per_inv_A(cfg), grid)
    imgs = synth.make_patterns(cfg, lib_np, idx)
    x = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    polar, norms, prof = tm.polar_transform(x, grid, lib=lib, **polar_kw)
    return lib, grid, imgs, polar, norms


def _window_bounds64(P_rows, rows, olib, pn):
    """float64 window bounds [T'] of one pattern from its compact polar rows."""
    n = olib.n_theta
    win = -(-n // 4)
    dl = 4 * win - n
    R = olib.R
    P = np.zeros((R, n))
    P[rows] = P_rows
    M = np.max(np.stack([np.roll(P, -d, axis=1) for d in range(min(win + dl, n))]), axis=0)
    M = np.maximum(M, 0.0)
    S = np.arange(4)[None, :]
    cols = (olib.K[:, None] + win * S - dl * (olib.K[:, None] // win + S >= 4)) % n
    vals = M[olib.J[:, None], cols] * (olib.Wt / olib.tnorm[olib.tid])[:, None]
    ub = np.zeros((olib.n_total, 4))
    np.add.at(ub, olib.tid, vals)
    return ub.max(axis=1) / pn


@pytest.mark.parametrize("case", ["plain", "gamma_subtract"])
def test_bounds_hold_and_equal_window_sums(tm, c1, c1_lib, case):
    kw = {} if case == "plain" else dict(gamma=0.5, subtract=0.05)
    _say("window bounds c1 B=48", case)
    lib, grid, imgs, polar, norms = _setup(tm, c1, c1_lib, range(48), **kw)
    ub = tm.bound_scores(lib, polar, norms).cpu().numpy()
    tt, ts, tq, bq, bs = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, 5,
                                                                  with_best=True))
    assert (ub >= bq).all(), float((bq - ub).max())
    olib = oracle.OracleLibrary.build(c1_lib, synth.px_per_inv_A(c1), c1.R, c1.n_theta)
    rows = np.unique(olib.J)                 # the touched rows, in compact order
    assert len(rows) == lib.rows()[0]
    P32 = polar.cpu().numpy().astype(np.float64)
    pn = norms.cpu().numpy()
    A = np.abs(P32).max(axis=(1, 2))
    wsum = np.zeros(olib.n_total)
    np.add.at(wsum, olib.tid, olib.Wt / olib.tnorm[olib.tid])
    cnt = np.bincount(olib.tid, minlength=olib.n_total)
    gam = cnt * 2.0 ** -24 / (1 - cnt * 2.0 ** -24)
    for b in range(len(imgs)):
        u64 = _window_bounds64(P32[b], rows, olib, pn[b])
        margin = gam * wsum * A[b] / pn[b]
        # at least the window sum; at most float16 rounding up of the window
        # maxima and the weights (2^-10 relative each) plus the float32 margins
        assert (ub[b] >= u64 * (1 - 1e-7)).all()
        assert (ub[b] <= u64 * (1 + 2.5e-3) + 2.5 * margin + 1e-12).all()


def test_bound_search_equals_plain_c1(tm, c1, c1_lib):
    import torch
    _say("bound search c1 B=64 (+ a blank and a rolled pattern)")
    lib, grid, imgs, polar, norms = _setup(tm, c1, c1_lib, range(64))
    # a blank pattern (zero norm: every template scores 0, scored in full)
    # and a pattern whose polar image is rolled by one column
    polar = torch.cat([polar, torch.zeros_like(polar[:1]), torch.roll(polar[3:4], 1, dims=2)])
    norms = torch.cat([norms, torch.zeros_like(norms[:1]), norms[3:4]])
    B = polar.shape[0]
    nr = torch.empty(B, dtype=torch.int32, device="cuda")
    for N in (1, 5, 17):
        pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, N))
        bt, bs, bq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, N,
                                                              coarse="bound", n_rescored=nr))
        assert np.array_equal(bt, pt) and np.array_equal(bs, ps)
        assert np.array_equal(bq, pq)
        n = nr.cpu().numpy()
        assert n[64] == lib.n_total                       # blank: every template
        assert (n[:64] >= N).all()
        if N <= 5:
            # deep ranks (N = 17 of 600 templates) sit among noise-level
            # scores that many bounds reach: full scans are legitimate there;
            # on 600 small templates a few patterns pass the 10% cap
            assert np.mean(n[:64] < lib.n_total) >= 0.75
        _say(f"N={N}: templates scored exactly per pattern: median {np.median(n[:64]):.0f}, "
             f"max {n[:64].max()} of {lib.n_total}")


def test_bound_search_c3_sample(tm):
    """The 20 000-template orthorhombic library: 256 patterns."""
    import torch
    cfg = synth.WORKLOADS[3]
    lib_np = synth.make_library(cfg)
    _say("bound search c3 B=256")
    lib, grid, imgs, polar, norms = _setup(tm, cfg, lib_np, range(0, 256 * 61, 61))
    nr = torch.empty(256, dtype=torch.int32, device="cuda")
    pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N))
    bt, bs, bq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N,
                                                          coarse="bound", n_rescored=nr))
    assert np.array_equal(bt, pt) and np.array_equal(bs, ps) and np.array_equal(bq, pq)
    n = nr.cpu().numpy()
    _say(f"templates scored exactly per pattern: mean {n.mean():.1f}, max {n.max()} of "
         f"{lib.n_total}")
    assert np.median(n) < 0.01 * lib.n_total


def test_bound_search_refusals(tm, c1, c1_lib):
    import torch
    grid = tm.PolarGrid(R=c1.R, n_theta=c1.n_theta, cx=c1.cx, cy=c1.cy)
    px = synth.px_per_inv_A(c1)
    neg = small_library(6, seed=3)
    neg["intensity"][2] = -0.5
    _say("bound search: negative weights, static entry, with a pre-filter")
    nlib = tm.Library(neg["kx"], neg["ky"], neg["intensity"], neg["offsets"], px, grid)
    p = torch.zeros((2, c1.R, c1.n_theta), dtype=torch.float32, device="cuda")
    nrm = torch.ones(2, dtype=torch.float64, device="cuda")
    with pytest.raises(tm.TMError) as e:
        tm.bound_scores(nlib, p, nrm)
    assert e.value.code == tm.TM_EUNSUPPORTED
    with pytest.raises(tm.TMError) as e:
        tm.match_batch(nlib, p, nrm, 3, coarse="bound")
    assert e.value.code == tm.TM_EUNSUPPORTED
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"], px, grid)
    o = tm._Opts(coarse=tm.TM_COARSE_BOUND)
    out = torch.empty((2, 5), dtype=torch.int32, device="cuda")
    r = tm._lib.tm_match_batch_static(lib._h, p.data_ptr(), nrm.data_ptr(), None, 2,
                                      ctypes.byref(o), 5, out.data_ptr(), out.data_ptr(),
                                      out.data_ptr(), None, None, None)
    assert r == tm.TM_EUNSUPPORTED
    o = tm._Opts(coarse=tm.TM_COARSE_BOUND, prefilter_keep=0.5)
    r = tm._lib.tm_match_batch(lib._h, p.data_ptr(), nrm.data_ptr(), p.data_ptr(), 2,
                               ctypes.byref(o), 5, out.data_ptr(), out.data_ptr(), out.data_ptr(),
                               None, None, None)
    assert r == tm.TM_EINVAL


@pytest.mark.parametrize("cap_frac", [0.004, 0.5])
def test_bound_search_split_passes_c2(tm, cap_frac):
    """The 4000-template library (1334 groups of 3), 192 patterns plus two
    blank ones and one with a non-finite norm. A cap of 0.4% of T' sends
    most patterns to full scans, each cut into several tasks whose partial
    lists are merged; a cap of 50% lets candidate lists grow past one task.
    Either way the result is the plain path's, bit for bit."""
    import torch
    cfg = synth.WORKLOADS[2]
    lib_np = synth.make_library(cfg)
    _say(f"bound search c2 B=195 cap_frac={cap_frac} (split passes)")
    lib, grid, imgs, polar, norms = _setup(tm, cfg, lib_np, range(0, 192 * 83, 83))
    polar = torch.cat([polar, torch.zeros_like(polar[:2]), polar[5:6].clone()])
    norms = torch.cat([norms, torch.zeros_like(norms[:2]), torch.full_like(norms[:1], float("nan"))])
    polar[-1, 0, 0] = float("nan")
    B = polar.shape[0]
    nr = torch.empty(B, dtype=torch.int32, device="cuda")
    pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N))
    bt, bs, bq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N, coarse="bound",
                                                          rescore_keep=cap_frac, n_rescored=nr))
    assert np.array_equal(bt, pt) and np.array_equal(bs, ps)
    assert np.array_equal(bq.view(np.int32), pq.view(np.int32))
    assert (pt[-1] == -1).all() and np.isnan(pq[-1]).all()
    n = nr.cpu().numpy()
    full = int((n == lib.n_total).sum())
    _say(f"full scans {full} of {B}; candidates per pattern max {n[n < lib.n_total].max()}")
    if cap_frac < 0.01:
        assert full >= B // 2
    else:
        assert n[n < lib.n_total].max() > 512


def test_bound_slots_order_equals_template_order(tm, c1, c1_lib):
    """tm_bound_scores_slots: the kernel's chunk-slot order with its slot map
    holds exactly tm_bound_scores' values; empty slots hold 0."""
    _say("bound slots vs template order, c1 B=16")
    lib, grid, imgs, polar, norms = _setup(tm, c1, c1_lib, range(16))
    ub = tm.bound_scores(lib, polar, norms).cpu().numpy()
    us, slots = tm.bound_scores_slots(lib, polar, norms)
    us = us.cpu().numpy()
    assert sorted(slots[slots >= 0].tolist()) == list(range(lib.n_total))
    assert np.array_equal(us[:, slots >= 0], ub[:, slots[slots >= 0]])
    assert (us[:, slots < 0] == 0).all()
    assert lib.bound_layout()["chunks"] * 64 == len(slots)


def _random_case(n_theta, seed, n_templates=40, R=48, H=104, W=100, B=12):
    """Small random library (up to 25 spots, duplicates merged) and patterns
    of rendered templates at random angles plus noise."""
    rng = np.random.default_rng(seed)
    lib = small_library(n_templates, seed, max_spots=25, g_min=0.08)
    px_per = (R - 4) / 1.2
    cx, cy = W / 2.0, H / 2.0
    yy, xx = np.mgrid[0:H, 0:W]
    imgs = np.zeros((B, H, W), dtype=np.float32)
    for b in range(B):
        t = int(rng.integers(0, n_templates))
        a, e = lib["offsets"][t], lib["offsets"][t + 1]
        phi = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(phi), np.sin(phi)
        img = 0.02 * rng.standard_normal((H, W))
        for kx, ky, w in zip(lib["kx"][a:e], lib["ky"][a:e], lib["intensity"][a:e]):
            x = cx + px_per * (c * kx - s * ky)
            y = cy + px_per * (s * kx + c * ky)
            img += w * np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * 1.5 ** 2))
        imgs[b] = img
    return lib, imgs, px_per, R, cx, cy


@pytest.mark.parametrize("n_theta", [64, 90, 181, 361, 720, 768])
def test_bound_search_theta_widths_layouts_and_sizes(tm, n_theta):
    """Windows of ceil(n_theta / 4) columns at other widths (the kernel with a
    runtime window stride; odd widths), full and compact polar layouts, N from
    1 to min(64, T'), B = 1 and B = 0: bounds hold and equal their window
    sums, the search equals the plain path bit for bit."""
    import torch
    _say(f"bound search, n_theta {n_theta}")
    lib_np, imgs, px_per, R, cx, cy = _random_case(n_theta, 300 + n_theta)
    grid = tm.PolarGrid(R=R, n_theta=n_theta, cx=cx, cy=cy)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px_per,
                     grid)
    assert lib.bound_layout()["win"] == -(-n_theta // 4)
    olib = oracle.OracleLibrary.build(lib_np, px_per, R, n_theta)
    x = torch.from_numpy(imgs).cuda()
    full, fnorms, _ = tm.polar_transform(x, grid)
    comp, cnorms, _ = tm.polar_transform(x, grid, lib=lib)
    ub_f = tm.bound_scores(lib, full, fnorms).cpu().numpy()
    ub_c = tm.bound_scores(lib, comp, cnorms).cpu().numpy()
    assert np.array_equal(ub_f, ub_c)
    best = tm.match_batch(lib, full, fnorms, 1, with_best=True)[3].cpu().numpy()
    assert (ub_f >= best).all(), float((best - ub_f).max())
    rows = np.unique(olib.J)
    P = full.cpu().numpy().astype(np.float64)
    pn = fnorms.cpu().numpy()
    A = np.abs(P[:, rows]).max(axis=(1, 2))
    wsum = np.zeros(olib.n_total)
    np.add.at(wsum, olib.tid, olib.Wt / olib.tnorm[olib.tid])
    cnt = np.bincount(olib.tid, minlength=olib.n_total) + 1
    gam = cnt * 2.0 ** -24 / (1 - cnt * 2.0 ** -24)
    for b in range(len(imgs)):
        u64 = _window_bounds64(P[b, rows], rows, olib, pn[b])
        assert (ub_f[b] >= u64 * (1 - 1e-7)).all()
        assert (ub_f[b] <= u64 * (1 + 2.5e-3) + 2.5 * gam * wsum * A[b] / pn[b] + 1e-12).all()
    Tp = lib.n_total
    for N in sorted({1, 4, min(64, Tp)}):
        for polar, norms in ((full, fnorms), (comp, cnorms)):
            pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, N))
            bt, bs, bq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, N,
                                                                  coarse="bound"))
            assert np.array_equal(bt, pt) and np.array_equal(bs, ps) and np.array_equal(bq, pq)
    # one pattern alone gives the same rows; an empty batch is a no-op
    b1 = [o.cpu().numpy()[0] for o in tm.match_batch(lib, comp[5:6].contiguous(),
                                                       cnorms[5:6].contiguous(), 4, coarse="bound")]
    ref = [o.cpu().numpy()[5] for o in tm.match_batch(lib, comp, cnorms, 4, coarse="bound")]
    assert all(np.array_equal(u, v) for u, v in zip(b1, ref))
    e = tm.match_batch(lib, comp[:0], cnorms[:0], 4, coarse="bound")
    assert e[0].shape == (0, 4)
