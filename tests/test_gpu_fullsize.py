"""GPU parity at the paper-scale sizes, in the launch configuration the
benchmark times: the whole scan (16 384 patterns of 256 x 256) through the
compact-row polar transform and one match launch, then sampled patterns
checked one by one against the FP64 oracle (Eq. 1 scores, top-N with the
index rule), properties checked on every pattern, and sampled patterns
re-run alone. Workloads: the 2000-template FCC library and the 20 000-
template orthorhombic library. Runs only on an MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
import synth
from parity import PatternRef, check_topn, oracle_best_pool, scores_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _properties(tt, ts, tq, Tp, n_theta):
    """Every pattern: valid ids and angles, finite scores in descending order,
    distinct templates."""
    assert ((tt >= 0) & (tt < Tp)).all()
    assert ((ts >= 0) & (ts < n_theta)).all()
    assert np.isfinite(tq).all()
    assert (np.diff(tq, axis=1) <= 0).all()
    assert (np.diff(np.sort(tt, axis=1), axis=1) > 0).all()


_SCANS = {}


@pytest.fixture(scope="module", autouse=True)
def _release_scans():
    """Drop the cached scan (several GiB of device memory) after the module."""
    yield
    _SCANS.clear()
    import torch
    torch.cuda.empty_cache()


def _scan(cid):
    """The whole scan of workload cid generated, uploaded, polar-transformed
    (compact rows, as the benchmark times it) and matched once; kept for the
    module's tests."""
    if cid in _SCANS:
        return _SCANS[cid]
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    _SCANS.clear()                       # one scan resident at a time
    cfg = synth.WORKLOADS[cid]
    _say("full scan", cid, cfg.B, "patterns", cfg.H, "x", cfg.W)
    lib_np = synth.make_library(cfg)
    imgs = synth.make_patterns_parallel(cfg, lib_np, cfg.B, workers=16)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    px = synth.px_per_inv_A(cfg)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, prof = tm.polar_transform(x, grid, lib=lib)
    top = [o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N)]
    _SCANS[cid] = dict(tm=tm, cfg=cfg, lib_np=lib_np, imgs=imgs, grid=grid, px=px, lib=lib, x=x,
                       polar=polar, norms=norms, prof=prof, top=top)
    return _SCANS[cid]


def test_full_scan_precision_forms():
    """FCC scan, precision form: the BF16 pre-filter path (keep 10 %) returns
    exact FP32 scores (sampled patterns against the oracle), and the Fourier
    route with certified rescoring returns exactly the plain path's top-N on
    every pattern."""
    sc = _scan(2)
    tm, cfg, lib_np, imgs, grid, px = (sc[k] for k in ("tm", "cfg", "lib_np", "imgs", "grid", "px"))
    lib, polar, norms, prof = sc["lib"], sc["polar"], sc["norms"], sc["prof"]
    tt, ts, tq = sc["top"]
    _say("BF16 pre-filter, keep 0.1, full scan")
    pt, ps, pq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N, profiles=prof,
                                                           prefilter_keep=0.1,
                                                           prefilter_prec="bf16"))
    _properties(pt, ps, pq, lib.info()["n_templates_total"], cfg.n_theta)
    olib = oracle.OracleLibrary.build(lib_np, px, cfg.R, cfg.n_theta)
    for b in (0, cfg.B - 1):
        ref = PatternRef(oracle.polar64(imgs[b].astype(np.float64), cfg.R, cfg.n_theta), olib)
        for t, s_, q in zip(pt[b], ps[b], pq[b]):
            assert scores_close(q, ref.best[int(t)]) and scores_close(q, ref.q_at(t, s_))
    _say("Fourier route, certified, full scan")
    flib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid,
                      fft=True)
    ft, fs, fq = (o.cpu().numpy() for o in tm.match_batch(flib, polar, norms, cfg.N, coarse="fft"))
    assert np.array_equal(ft, tt) and np.array_equal(fs, ts)
    assert scores_close(fq, tq).all()


@pytest.mark.parametrize("cid,n_sample", [(2, 10)])
def test_full_scan_sampled_against_oracle(cid, n_sample):
    sc = _scan(cid)
    tm, cfg, lib_np, imgs, grid, px, lib, x = (sc[k] for k in
                                              ("tm", "cfg", "lib_np", "imgs", "grid", "px", "lib", "x"))
    B = cfg.B
    tt, ts, tq = sc["top"]
    Tp = lib.info()["n_templates_total"]
    _say("layout", lib.layout(), "Tp", Tp)
    _properties(tt, ts, tq, Tp, cfg.n_theta)

    rng = np.random.default_rng(100 + cid)
    fixed = [B - 1, 0, B // 2][:n_sample]
    extra = rng.choice(np.arange(1, B - 1), max(0, n_sample - len(fixed)), replace=False).tolist()
    sample = sorted(set(fixed + extra))
    olib = oracle.OracleLibrary.build(lib_np, px, cfg.R, cfg.n_theta)
    for b in sample:
        _say("oracle check, pattern", b)
        ref = PatternRef(oracle.polar64(imgs[b].astype(np.float64), cfg.R, cfg.n_theta), olib)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4)

    # the same patterns alone give the same results as inside the scan
    for b in sample[:2]:
        p1, n1, _ = tm.polar_transform(x[b:b + 1].contiguous(), grid, lib=lib)
        t1, s1, q1 = (o.cpu().numpy()[0] for o in tm.match_batch(lib, p1, n1, cfg.N))
        assert np.array_equal(t1, tt[b]) and np.array_equal(s1, ts[b]) and np.array_equal(q1, tq[b])



def test_c3_scan_sampled_against_oracle_pool():
    """The 20 000-template orthorhombic scan (16 384 patterns): 32 sampled
    patterns (the first, the last and 30 drawn at random) against the oracle's
    exact search, spread over 16 worker processes (about half a minute per
    pattern each)."""
    sc = _scan(3)
    cfg, lib_np, imgs, px, lib = (sc[k] for k in ("cfg", "lib_np", "imgs", "px", "lib"))
    tt, ts, tq = sc["top"]
    B = cfg.B
    _properties(tt, ts, tq, lib.info()["n_templates_total"], cfg.n_theta)
    rng = np.random.default_rng(303)
    sample = sorted({0, B - 1, *rng.choice(np.arange(1, B - 1), 30, replace=False).tolist()})
    _say("C3 oracle pool over", len(sample), "patterns")
    bests = oracle_best_pool(3, [imgs[b] for b in sample], workers=16)
    olib = oracle.OracleLibrary.build(lib_np, px, cfg.R, cfg.n_theta)
    exact = 0
    for b, (best, arg) in zip(sample, bests):
        ref = PatternRef(oracle.polar64(imgs[b].astype(np.float64), cfg.R, cfg.n_theta), olib,
                         best=best, arg=arg)
        exact += check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4)
    _say("ranks checked exactly:", exact, "of", len(sample) * cfg.N)
    assert exact >= len(sample)          # at least the top-1 of a typical pattern


def test_c3_scan_bound_search_and_reduced_precision():
    """On the whole 20 000-template scan: the exact search with window bounds
    returns the plain path's top-N bit for bit on every pattern, and the
    reduced-precision pre-filter paths (keep 10 %) agree with the plain
    path's top-1 on at least 99 % (BF16, FP16) and 98 % (FP8) of patterns."""
    import torch
    sc = _scan(3)
    tm, cfg, lib, polar, norms, prof = (sc[k] for k in ("tm", "cfg", "lib", "polar", "norms", "prof"))
    tt, ts, tq = sc["top"]
    _say("C3 bound search, whole scan")
    nr = torch.empty(cfg.B, dtype=torch.int32, device="cuda")
    bt, bs, bq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N, coarse="bound",
                                                          n_rescored=nr))
    assert np.array_equal(bt, tt) and np.array_equal(bs, ts) and np.array_equal(bq, tq)
    n = nr.cpu().numpy()
    _say("templates scored exactly: mean", float(n.mean()), "full scans", int((n == lib.n_total).sum()))
    for prec, floor in (("bf16", 0.99), ("fp16", 0.99), ("fp8", 0.98)):
        pt = tm.match_batch(lib, polar, norms, cfg.N, profiles=prof, prefilter_keep=0.1,
                            prefilter_prec=prec)[0].cpu().numpy()
        agree = float(np.mean(pt[:, 0] == tt[:, 0]))
        _say(prec, "keep 0.1 top-1 agreement with the plain path", agree)
        assert agree >= floor
