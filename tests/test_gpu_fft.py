"""GPU parity of the Fourier-route coarse scorer and its rescoring.

* tm_fft_scores: every approximate per-template best score lies within the
  library's certified bound of the FP64 oracle's exact best score (plus the
  polar stage's own float32 tolerance); the approximate angle is a shift
  whose exact score is within twice that of the best, and equals the
  oracle's wherever the oracle's angle margin exceeds 1e-4;
* certified rescoring: the top-N equals the oracle's (margin rule) and the
  plain float32 path's;
* keep-fraction rescoring: every returned entry is an exact score;
* the bound the library reports equals the one derived independently in
  tests/fft_bound.py.
Runs only on an MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import small_library
from fft_bound import fft16_error_bound
from parity import PatternRef, check_topn, scores_close

pytestmark = pytest.mark.gpu

POLAR_SLACK = 2e-5     # effect of the float32 polar image on Q (polar parity)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _say(*a):
    print("[case]", *a, flush=True)


def _row_and_max(olib):
    """(touched polar rows, most pixels of one template in one row, most
    pixels of one template)."""
    key = olib.tid * olib.R + olib.J
    row_max = int(np.bincount(key).max()) if len(key) else 1
    return max(1, len(np.unique(olib.J))), row_max, int(np.diff(olib.starts).max())


def _lib(tm, lib_np, cfg_or_grid, px_per, **kw):
    grid = cfg_or_grid
    if not isinstance(grid, tm.PolarGrid):
        grid = tm.PolarGrid(R=grid.R, n_theta=grid.n_theta, cx=grid.cx, cy=grid.cy)
    return tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px_per,
                      grid, fft=True, **kw), grid


def _polar(tm, imgs, grid):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    return tm.polar_transform(x, grid)


def _check_scores(q, a, imgs, olib, R, n_theta, eps, cx=None, cy=None):
    """Approximate scores within eps of the oracle; angles where unique."""
    worst = 0.0
    n_ang = 0
    for b in range(len(imgs)):
        P = oracle.polar64(imgs[b], R, n_theta, cx=cx, cy=cy)
        Q = oracle.scores64(P, olib)
        best = Q.max(axis=1)
        err = np.abs(q[b].astype(np.float64) - best)
        worst = max(worst, float(err.max()))
        assert err.max() <= eps + POLAR_SLACK, (b, float(err.max()), eps)
        if a is not None:
            # the approximate angle is a near-maximum within the bound ...
            at = Q[np.arange(len(best)), a[b].astype(np.int64)]
            assert (at >= best - 2.0 * (eps + POLAR_SLACK)).all(), b
            # ... and the oracle's wherever its angle margin exceeds the
            # contract margin of 1e-4 (far above the errors observed)
            srt = np.sort(Q, axis=1)
            margin = srt[:, -1] - srt[:, -2]
            sure = margin > 1e-4
            assert np.array_equal(a[b][sure], Q.argmax(axis=1)[sure]), b
            n_ang += int(sure.sum())
    return worst, n_ang


def test_bound_value_matches_derivation(tm, c1, c1_lib, c1_olib):
    _say("fft bound c1")
    lib, _ = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    n_rows, row_max, n_max = _row_and_max(c1_olib)
    assert n_rows == lib.rows()[0]
    ref = fft16_error_bound(n_rows, c1.n_theta, row_max, n_max)
    assert abs(lib.fft_error_bound() - ref) <= 1e-12 * ref
    assert lib.fft_error_bound() < 2.5e-3


def test_fft_scores_c1(tm, c1, c1_lib, c1_olib):
    _say("fft scores c1 B=64")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = synth.make_patterns(c1, c1_lib, range(64))
    polar, norms, _ = _polar(tm, imgs, grid)
    q, a = tm.fft_scores(lib, polar, norms)
    torch.cuda.synchronize()
    eps = lib.fft_error_bound()
    worst, n_ang = _check_scores(q.cpu().numpy(), a.cpu().numpy(), imgs, c1_olib, c1.R,
                                 c1.n_theta, eps)
    _say(f"max |Q~ - Q| = {worst:.3e}, bound {eps:.3e}, angles checked {n_ang}")
    assert n_ang > 64 * 50


def test_certified_c1_equals_oracle_and_plain(tm, c1, c1_lib, c1_olib):
    _say("fft certified c1 B=64 N=5")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = synth.make_patterns(c1, c1_lib, range(64))
    polar, norms, _ = _polar(tm, imgs, grid)
    nr = torch.empty(64, dtype=torch.int32, device="cuda")
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, 5, coarse="fft",
                                                          n_rescored=nr))
    pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, 5))
    nr = nr.cpu().numpy()
    for b in range(64):
        ref = PatternRef(oracle.polar64(imgs[b], c1.R, c1.n_theta), c1_olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4)
    assert np.array_equal(tt, pt) and np.array_equal(ts, ps)
    assert np.allclose(tq, pq, rtol=0, atol=2e-6)
    assert (nr >= 5).all() and (nr <= lib.n_total).all()
    _say(f"rescored per pattern: mean {nr.mean():.1f}, max {nr.max()} of {lib.n_total}")


def test_keep_policy_c1_entries_are_exact(tm, c1, c1_lib, c1_olib):
    _say("fft keep 0.25 c1 B=32")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = synth.make_patterns(c1, c1_lib, range(100, 132))
    polar, norms, _ = _polar(tm, imgs, grid)
    nr = torch.empty(32, dtype=torch.int32, device="cuda")
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(
        lib, polar, norms, 5, coarse="fft", rescore="keep", rescore_keep=0.25, n_rescored=nr))
    assert (nr.cpu().numpy() == int(np.ceil(0.25 * lib.n_total))).all()
    eps = lib.fft_error_bound()
    for b in range(32):
        ref = PatternRef(oracle.polar64(imgs[b], c1.R, c1.n_theta), c1_olib)
        assert len(set(tt[b].tolist())) == 5
        for t, s, q in zip(tt[b], ts[b], tq[b]):
            assert scores_close(q, ref.best[int(t)])
            assert scores_close(q, ref.q_at(t, s))
        o0, o1 = ref.order[0], ref.order[1]
        if ref.best[o0] - ref.best[o1] > 2.0 * (eps + POLAR_SLACK):
            assert int(tt[b, 0]) == int(ref.ids[o0])


def _synthetic_case(n_theta, seed, n_templates=40, R=48, H=104, W=100):
    rng = np.random.default_rng(seed)
    lib = small_library(n_templates, seed, max_spots=25, g_min=0.08)
    px_per = (R - 4) / 1.2
    cx, cy = W / 2.0, H / 2.0
    yy, xx = np.mgrid[0:H, 0:W]
    imgs = np.zeros((5, H, W), dtype=np.float32)
    for b in range(5):
        t = int(rng.integers(0, n_templates))
        a, bnd = lib["offsets"][t], lib["offsets"][t + 1]
        phi = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(phi), np.sin(phi)
        img = 0.02 * rng.standard_normal((H, W))
        for kx, ky, w in zip(lib["kx"][a:bnd], lib["ky"][a:bnd], lib["intensity"][a:bnd]):
            x = cx + px_per * (c * kx - s * ky)
            y = cy + px_per * (s * kx + c * ky)
            img += w * np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * 1.5 ** 2))
        imgs[b] = img
    return lib, imgs, px_per, R, cx, cy


@pytest.mark.parametrize("n_theta", [90, 180, 360, 720])
def test_theta_widths(tm, n_theta):
    _say(f"fft theta width {n_theta}")
    import torch
    lib_np, imgs, px_per, R, cx, cy = _synthetic_case(n_theta, 100 + n_theta)
    grid = tm.PolarGrid(R=R, n_theta=n_theta, cx=cx, cy=cy)
    lib, _ = _lib(tm, lib_np, grid, px_per)
    olib = oracle.OracleLibrary.build(lib_np, px_per, R, n_theta)
    n_rows, row_max, n_max = _row_and_max(olib)
    eps = lib.fft_error_bound()
    assert abs(eps - fft16_error_bound(n_rows, n_theta, row_max, n_max)) <= 1e-12 * eps
    polar, norms, _ = _polar(tm, imgs, grid)
    q, a = tm.fft_scores(lib, polar, norms)
    tt, ts, tq = tm.match_batch(lib, polar, norms, 4, coarse="fft")
    torch.cuda.synchronize()
    worst, _ = _check_scores(q.cpu().numpy(), a.cpu().numpy(), imgs, olib, R, n_theta, eps,
                             cx=cx, cy=cy)
    _say(f"max |Q~ - Q| = {worst:.3e}, bound {eps:.3e}")
    tt, ts, tq = tt.cpu().numpy(), ts.cpu().numpy(), tq.cpu().numpy()
    for b in range(len(imgs)):
        ref = PatternRef(oracle.polar64(imgs[b], R, n_theta, cx=cx, cy=cy), olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4)


def test_batch_independence_and_ragged_sizes(tm, c1, c1_lib):
    """A pattern's approximate scores do not depend on its batch (sizes 1, 65,
    130: ragged tiles of 32 and 64 patterns)."""
    _say("fft batch independence c1")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = synth.make_patterns(c1, c1_lib, range(130))
    polar, norms, _ = _polar(tm, imgs, grid)
    q_all, a_all = tm.fft_scores(lib, polar, norms)
    for lo, hi in ((7, 8), (0, 65), (65, 130)):
        q, a = tm.fft_scores(lib, polar[lo:hi].contiguous(), norms[lo:hi].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(q, q_all[lo:hi]) and torch.equal(a, a_all[lo:hi]), (lo, hi)
    tt, ts, tq = tm.match_batch(lib, polar[:1].contiguous(), norms[:1].contiguous(), 5,
                                coarse="fft")
    pt, ps, pq = tm.match_batch(lib, polar[:1].contiguous(), norms[:1].contiguous(), 5)
    assert torch.equal(tt, pt) and torch.equal(ts, ps)


def test_zero_pattern_and_errors(tm, c1, c1_lib):
    _say("fft degenerate inputs")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = np.zeros((3, c1.H, c1.W), dtype=np.float32)
    polar, norms, _ = _polar(tm, imgs, grid)
    q, a = tm.fft_scores(lib, polar, norms)
    assert torch.count_nonzero(q).item() == 0
    nr = torch.empty(3, dtype=torch.int32, device="cuda")
    tt, ts, tq = tm.match_batch(lib, polar, norms, 5, coarse="fft", n_rescored=nr)
    assert torch.count_nonzero(tq).item() == 0
    assert tt.cpu().numpy().tolist() == [[0, 1, 2, 3, 4]] * 3     # all ties: lowest indices
    assert (nr.cpu().numpy() == lib.n_total).all()               # certified set too large: full scan
    plain = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                       synth.px_per_inv_A(c1), grid)
    with pytest.raises(tm.TMError):
        tm.fft_scores(plain, polar, norms)
    with pytest.raises(tm.TMError):
        tm.match_batch(plain, polar, norms, 5, coarse="fft")
    with pytest.raises(tm.TMError):
        tm.match_batch(lib, polar, norms, 5, coarse="fft", rescore="keep")   # keep fraction 0


def test_compact_rows_equal_full(tm, c1, c1_lib):
    """The Fourier route on a polar image holding only the library's touched
    rows gives bit-identical scores and top-N to the full image."""
    _say("fft compact rows c1")
    import torch
    lib, grid = _lib(tm, c1_lib, c1, synth.px_per_inv_A(c1))
    imgs = synth.make_patterns(c1, c1_lib, range(40))
    x = torch.from_numpy(imgs).cuda()
    polar, norms, _ = tm.polar_transform(x, grid)
    cpolar, cnorms, _ = tm.polar_transform(x, grid, lib=lib)
    assert cpolar.shape[1] == lib.rows()[0] < c1.R
    q, a = tm.fft_scores(lib, polar, norms)
    cq, ca = tm.fft_scores(lib, cpolar, cnorms)
    assert torch.equal(q, cq) and torch.equal(a, ca)
    full = tm.match_batch(lib, polar, norms, 5, coarse="fft")
    comp = tm.match_batch(lib, cpolar, cnorms, 5, coarse="fft")
    for u, v in zip(full, comp):
        assert torch.equal(u, v)
