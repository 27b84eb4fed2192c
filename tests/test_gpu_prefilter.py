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


# ---- the reduced-precision kept sets, emulated on the CPU -------------------
# The kernel's arithmetic, restated from its definition (not from its code):
# template profiles are the library's summed pixel weights per polar row,
# normalised to unit length and rounded to float32; a pattern profile is
# scaled by 1 / max|profile| (float32 division and product); operands are
# rounded to bfloat16 or float16 (round to nearest even) or, for FP8, each
# template profile is first scaled by 1 / its maximum and both operands are
# rounded to OCP e4m3 (3 mantissa bits, exponent bias 7, subnormal quantum
# 2^-9, round to nearest even) and the product is scaled back by the template
# maximum; products of the rounded operands accumulate in float32. The
# emulation sums in float64, so kept sets may differ only by templates whose
# score ties the n_keep-th at float32 accumulation level: a sum of R
# non-negative terms in float32 is within gamma_R ~ R 2^-24 of the exact one.

def _f32_profiles(olib):
    prof = oracle.radial_profiles64(olib)
    nrm = np.sqrt((prof * prof).sum(axis=1, keepdims=True))
    out = np.zeros_like(prof)
    np.divide(prof, nrm, out=out, where=nrm > 0)
    return out.astype(np.float32)


def _bf16(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _e4m3(x, bias=7):
    """Non-negative x to the nearest e4m3 value (ties to even): OCP e4m3fn
    (bias 7) or, for comparison, the bias-8 variant."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x > 0
    e = np.floor(np.log2(x[nz]))
    emin = 1 - bias
    q = np.where(e < emin, 2.0 ** (emin - 3), 2.0 ** (e - 3))
    out[nz] = np.rint(x[nz] / q) * q
    return out


def _emulated_scores(prec, profT32, profP32, fp8_bias=7):
    """Scores [B, T] as the kernel forms them (float64 sums)."""
    x = profP32.T                                        # [B, R] float32
    if prec == "fp32":
        return x.astype(np.float64) @ profT32.T.astype(np.float64)
    m = np.abs(x).max(axis=1)
    ps = np.where(m > 0, np.float32(1.0) / np.where(m > 0, m, np.float32(1.0)), np.float32(1.0))
    xs = (x * ps[:, None].astype(np.float32)).astype(np.float32)
    if prec == "bf16":
        return _bf16(xs) @ _bf16(profT32).T
    if prec == "fp16":
        return xs.astype(np.float16).astype(np.float64) @ profT32.astype(np.float16).astype(np.float64).T
    tmax = np.abs(profT32).max(axis=1)
    ts = np.where(tmax > 0, np.float32(1.0) / np.where(tmax > 0, tmax, np.float32(1.0)),
                  np.float32(1.0)).astype(np.float32)
    a = (profT32 * ts[:, None]).astype(np.float32)
    S = _e4m3(xs, fp8_bias) @ _e4m3(a, fp8_bias).T
    return S * np.where(tmax > 0, tmax, 1.0).astype(np.float64)[None, :]


def _kept_equal_up_to_ties(kept, S, n_keep, rel=2e-5):
    """GPU kept set (ascending ids) vs the emulated scores of one pattern:
    identical except templates within rel of the n_keep-th score."""
    kept = np.asarray(kept)
    assert len(set(kept.tolist())) == n_keep and np.all(np.diff(kept) > 0)
    order = np.lexsort((np.arange(len(S)), -S))
    thr = S[order[n_keep - 1]]
    diff = set(kept.tolist()) ^ set(order[:n_keep].tolist())
    bad = [t for t in diff if abs(S[t] - thr) > rel * abs(thr) + 1e-12]
    return bad, len(diff)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp8"])
def test_prefilter_kept_sets_emulated(tm, prec):
    """32 patterns of the 20 000-template scan, pattern profiles from the
    oracle (rounded to float32) as the pre-filter's input: the GPU kept sets
    (keep 10 %) equal the emulated ones up to float32-level ties."""
    import torch
    cfg = synth.WORKLOADS[3]
    lib_np = synth.make_library(cfg)
    idx = list(range(0, cfg.B, cfg.B // 32))
    _say("prefilter", prec, "emulated, config 3, patterns", len(idx))
    imgs = synth.make_patterns(cfg, lib_np, idx)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    px = synth.px_per_inv_A(cfg)
    tml = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid)
    olib = oracle.OracleLibrary.build(lib_np, px, cfg.R, cfg.n_theta)
    profP = np.stack([oracle.profile64(oracle.polar64(im.astype(np.float64), cfg.R, cfg.n_theta))
                      for im in imgs], axis=1).astype(np.float32)          # [R, B]
    n_keep = math.ceil(0.1 * olib.T_base)
    kept = tm.prefilter(tml, torch.from_numpy(profP).cuda(), n_keep, prec).cpu().numpy()
    profT = _f32_profiles(olib)
    S = _emulated_scores(prec, profT, profP)
    n_diff = 0
    for b in range(len(idx)):
        bad, nd = _kept_equal_up_to_ties(kept[b], S[b], n_keep)
        if bad and prec == "fp8":
            alt, _ = _kept_equal_up_to_ties(kept[b], _emulated_scores(prec, profT, profP, 8)[b], n_keep)
            _say("fp8 pattern", idx[b], "mismatches (bias 7)", len(bad), "(bias 8)", len(alt))
        assert not bad, (prec, idx[b], bad[:5])
        n_diff += nd
    _say(prec, "kept-set entries differing at tie level:", n_diff, "of", n_keep * len(idx))


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
