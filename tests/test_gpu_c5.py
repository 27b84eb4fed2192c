"""GPU parity on the large multi-phase library (50 000 templates: FCC, HCP,
orthorhombic; 100 000 with mirrors; uint16 Poisson patterns; top-10):
plain path against the FP64 oracle on 8 sampled patterns, and the FP8
pre-filter path's entries are exact scores. Runs only on an MI355X."""
import numpy as np
import pytest

import oracle
import synth
from parity import PatternRef, check_topn, oracle_best_pool, scores_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def c5():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    cfg = synth.WORKLOADS[5]
    lib_np = synth.make_library(cfg)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    px = synth.px_per_inv_A(cfg)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid)
    olib = oracle.OracleLibrary.build(lib_np, px, cfg.R, cfg.n_theta)
    idx = [0, 17, 1023, 65536, 130000, 200000, 250001, 262143]
    imgs = synth.make_patterns(cfg, lib_np, idx)
    x = torch.from_numpy(imgs.view(np.int16)).cuda()
    polar, norms, prof = tm.polar_transform(x, grid)
    return tm, cfg, lib, olib, idx, imgs, polar, norms, prof


def test_c5_plain_matches_oracle(c5):
    """8 patterns spread over the scan against the oracle's exact search
    (about 40 s per pattern; one worker process per pattern)."""
    tm, cfg, lib, olib, idx, imgs, polar, norms, prof = c5
    _say("C5 plain", idx, "layout", lib.layout())
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N))
    bests = oracle_best_pool(5, list(imgs), workers=len(idx))
    for b, (best, arg) in enumerate(bests):
        ref = PatternRef(oracle.polar64(imgs[b].astype(np.float64), cfg.R, cfg.n_theta), olib,
                         best=best, arg=arg)
        check_topn(ref, tt[b], ts[b], tq[b], margin=1e-4)


def test_c5_fp8_prefilter_entries_exact(c5):
    tm, cfg, lib, olib, idx, imgs, polar, norms, prof = c5
    _say("C5 fp8 pre-filter", idx)
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(
        lib, polar, norms, cfg.N, profiles=prof, prefilter_keep=0.1, prefilter_prec="fp8"))
    pt = tm.match_batch(lib, polar, norms, cfg.N)[0].cpu().numpy()
    b = 1
    ref = PatternRef(oracle.polar64(imgs[b].astype(np.float64), cfg.R, cfg.n_theta), olib)
    for t, s, q in zip(tt[b], ts[b], tq[b]):
        assert scores_close(q, ref.best[int(t)]) and scores_close(q, ref.q_at(t, s))
    _say("top-1 agreement fp8 vs plain", float(np.mean(tt[:, 0] == pt[:, 0])))
