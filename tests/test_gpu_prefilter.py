"""GPU parity of the pre-filter (Section 2.2, Fig. 3) and of candidate
rescoring against the FP64 oracle. Marked gpu."""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import small_library
from parity import PatternRef, check_topn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _say(*a):
    print("[case]", *a, flush=True)


def _setup(tm, cid, idx, grouping=True):
    import torch
    cfg = synth.WORKLOADS[cid]
    lib = synth.make_library(cid)
    imgs = synth.make_patterns(cfg, lib, idx)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    px = synth.px_per_inv_A(cfg)
    tml = tm.Library(lib["kx"], lib["ky"], lib["intensity"], lib["offsets"], px, grid,
                     grouping=grouping)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, prof = tm.polar_transform(x, grid)
    olib = oracle.OracleLibrary.build(lib, px, cfg.R, cfg.n_theta)
    return cfg, lib, imgs, tml, polar, norms, prof, olib


def _oracle_cos(olib, P):
    profT = oracle.radial_profiles64(olib)
    _, cos = oracle.prefilter64(oracle.profile64(P), profT, 1.0)
    return cos


def _check_kept(kept, cos, n_keep, tol):
    """GPU kept set vs the oracle's cosines: identical except for templates
    whose cosine is within tol of the boundary (the n_keep-th cosine)."""
    kept = np.asarray(kept)
    assert len(set(kept.tolist())) == n_keep and np.all(np.diff(kept) > 0)
    order = np.lexsort((np.arange(len(cos)), -cos))
    ref = set(order[:n_keep].tolist())
    thr = cos[order[n_keep - 1]]
    for t in set(kept.tolist()) ^ ref:
        assert abs(cos[t] - thr) <= tol, (t, cos[t], thr)
    return len(set(kept.tolist()) & ref) / n_keep


@pytest.mark.parametrize("cid,n", [(1, 16), (3, 4)])
def test_prefilter_fp32_kept_sets(tm, cid, n):
    idx = list(range(0, 64, 64 // n)) if cid == 1 else [0, 4096, 8192, 16383]
    _say("prefilter fp32 kept sets config", cid, "patterns", idx)
    cfg, lib, imgs, tml, polar, norms, prof, olib = _setup(tm, cid, idx)
    n_keep = math.ceil(0.1 * olib.T_base)
    kept = tm.prefilter(tml, prof, n_keep, "fp32").cpu().numpy()
    for b in range(len(idx)):
        P = oracle.polar64(imgs[b], cfg.R, cfg.n_theta)
        _check_kept(kept[b], _oracle_cos(olib, P), n_keep, tol=2e-5)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_prefilter_reduced_precision_overlap(tm, prec):
    idx = [0, 4096, 8192, 16383]
    _say("prefilter", prec, "config 3", idx)
    cfg, lib, imgs, tml, polar, norms, prof, olib = _setup(tm, 3, idx)
    n_keep = math.ceil(0.1 * olib.T_base)
    kept = tm.prefilter(tml, prof, n_keep, prec).cpu().numpy()
    # error bound of the reduced-precision cosine: unit roundoff of the
    # format times a small constant (profiles are non-negative)
    tol = {"bf16": 2e-2, "fp16": 4e-3, "fp8": 1.5e-1}[prec]
    for b in range(len(idx)):
        P = oracle.polar64(imgs[b], cfg.R, cfg.n_theta)
        frac = _check_kept(kept[b], _oracle_cos(olib, P), n_keep, tol=tol)
        _say(prec, "pattern", idx[b], "kept-set agreement", round(frac, 4))


def test_prefiltered_match_equals_oracle_on_kept(tm):
    """tm_match_batch with a pre-filter = exact top-N over the kept templates
    and their mirrors (oracle restricted to the GPU's kept set), and the kept
    set matches the oracle's pre-filter."""
    import torch
    idx = list(range(0, 64, 4))
    cfg, lib, imgs, tml, polar, norms, prof, olib = _setup(tm, 1, idx)
    n_keep = math.ceil(0.1 * olib.T_base)
    _say("prefiltered match config 1", len(idx), "patterns, keep", n_keep)
    tt, ts, tq = tm.match_batch(tml, polar, norms, cfg.N, profiles=prof, prefilter_keep=0.1,
                                prefilter_prec="fp32")
    kept = tm.prefilter(tml, prof, n_keep, "fp32").cpu().numpy()
    tt, ts, tq = tt.cpu().numpy(), ts.cpu().numpy(), tq.cpu().numpy()
    for b in range(len(idx)):
        P = oracle.polar64(imgs[b], cfg.R, cfg.n_theta)
        _check_kept(kept[b], _oracle_cos(olib, P), n_keep, tol=2e-5)
        ids = np.sort(np.concatenate([kept[b], kept[b] + olib.T_base]))
        ref = PatternRef(P, olib, templates=ids)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)


@pytest.mark.parametrize("grouping", [True, False])
def test_keep_all_equals_full_path(tm, grouping):
    idx = list(range(8))
    cfg, lib, imgs, tml, polar, norms, prof, olib = _setup(tm, 1, idx, grouping=grouping)
    _say("keep = 1 vs full path, grouping", grouping)
    full = [o.cpu().numpy() for o in tm.match_batch(tml, polar, norms, cfg.N)]
    pre = [o.cpu().numpy() for o in tm.match_batch(tml, polar, norms, cfg.N, profiles=prof,
                                                   prefilter_keep=1.0)]
    assert np.array_equal(full[0], pre[0]) and np.array_equal(full[1], pre[1])
    # scores agree to the float32 summation-order difference between the
    # grouped and per-template record layouts
    assert np.allclose(full[2], pre[2], rtol=2e-6, atol=1e-9)


def test_match_candidates_explicit_lists(tm):
    import torch
    R, nt, px = 40, 180, 33.0
    lib = small_library(60, seed=7, max_spots=12, g_max=1.1, g_min=0.3)
    olib = oracle.OracleLibrary.build(lib, px, R, nt)
    grid = tm.PolarGrid(R=R, n_theta=nt, cx=48.0, cy=48.0)
    tml = tm.Library(lib["kx"], lib["ky"], lib["intensity"], lib["offsets"], px, grid)
    rng = np.random.default_rng(8)
    imgs = rng.random((5, 96, 96)).astype(np.float32)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, _ = tm.polar_transform(x, grid)
    n_cand = 25
    cand = np.stack([rng.choice(olib.n_total, n_cand, replace=False) for _ in range(5)])
    cand[1, 3] = -1            # ignored entries
    cand[2, 7] = olib.n_total  # out of range: ignored
    _say("explicit candidates", cand.shape)
    tt, ts, tq = tm.match_candidates(tml, polar, norms, torch.from_numpy(cand.astype(np.int32)).cuda(), 6)
    tt, ts, tq = tt.cpu().numpy(), ts.cpu().numpy(), tq.cpu().numpy()
    for b in range(5):
        ids = np.sort([c for c in cand[b] if 0 <= c < olib.n_total])
        P = oracle.polar64(imgs[b], R, nt, cx=48.0, cy=48.0)
        ref = PatternRef(P, olib, templates=ids)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4, tight=True)
