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
from parity import PatternRef, check_topn

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


# the oracle's exact search over 40 000 templates takes about half a minute
# per pattern on one core: one sampled pattern (the scan's last) for C3
@pytest.mark.parametrize("cid,n_sample", [(2, 10), (3, 1)])
def test_full_scan_sampled_against_oracle(cid, n_sample):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    cfg = synth.CONFIGS[cid]
    B = cfg.B
    _say("full scan", cid, B, "patterns", cfg.H, "x", cfg.W)
    lib_np = synth.make_library(cfg)
    imgs = synth.make_patterns_parallel(cfg, lib_np, B, workers=16)
    grid = tm.PolarGrid(R=cfg.R, n_theta=cfg.n_theta, cx=cfg.cx, cy=cfg.cy)
    px = synth.px_per_inv_A(cfg)
    lib = tm.Library(lib_np["kx"], lib_np["ky"], lib_np["intensity"], lib_np["offsets"], px, grid)
    x = torch.from_numpy(imgs).cuda()
    polar, norms, _ = tm.polar_transform(x, grid, lib=lib)
    tt, ts, tq = (o.cpu().numpy() for o in tm.match_batch(lib, polar, norms, cfg.N))
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
