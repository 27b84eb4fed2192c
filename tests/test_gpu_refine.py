"""GPU parity of the sub-bin in-plane angle (tm_refine_angles) against the
oracle's refine_angle64 on the oracle's own top-N: wherever the GPU reports
the oracle's template and shift, the refined angles agree within the effect
of the score tolerance on the parabola's vertex. Runs only on an MI355X."""
import numpy as np
import pytest

import oracle
import synth
from parity import PatternRef

pytestmark = pytest.mark.gpu


def test_refined_angles_c1(c1, c1_lib, c1_olib):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    print("[case] refine angles c1 B=32 N=5 (full and compact polar)", flush=True)
    grid = tm.PolarGrid(R=c1.R, n_theta=c1.n_theta, cx=c1.cx, cy=c1.cy)
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                     synth.px_per_inv_A(c1), grid)
    imgs = synth.make_patterns(c1, c1_lib, range(32))
    x = torch.from_numpy(imgs).cuda()
    polar, norms, _ = tm.polar_transform(x, grid)
    cpolar, cnorms, _ = tm.polar_transform(x, grid, lib=lib)
    tt, ts, tq = tm.match_batch(lib, polar, norms, 5)
    ref_deg = tm.refine_angles(lib, polar, norms, tt, ts).cpu().numpy()
    cmp_deg = tm.refine_angles(lib, cpolar, cnorms, tt, ts).cpu().numpy()
    assert np.array_equal(ref_deg, cmp_deg)
    tt, ts = tt.cpu().numpy(), ts.cpu().numpy()
    step = 360.0 / c1.n_theta
    checked = 0
    for b in range(len(imgs)):
        P = oracle.polar64(imgs[b], c1.R, c1.n_theta)
        ref = PatternRef(P, c1_olib)
        for r in range(5):
            t = int(ref.ids[ref.order[r]])
            s = int(ref.arg[ref.order[r]])
            if int(tt[b, r]) != t or int(ts[b, r]) != s:
                continue
            Q = ref.Q[ref._pos[t]]
            qm, q0, qp = Q[(s - 1) % c1.n_theta], Q[s], Q[(s + 1) % c1.n_theta]
            den = qm - 2 * q0 + qp
            if den > -1e-6:
                continue                       # vertex test too close to call
            want = oracle.refine_angle64(P, c1_olib, t, s)
            tol = step * (4.0 * max(1e-5 * abs(q0), 1e-7) / abs(den) + 1e-4)
            got = float(ref_deg[b, r])
            assert abs((got - want + 180.0) % 360.0 - 180.0) <= tol, (b, r, got, want, tol)
            checked += 1
    print(f"[case] refined angles checked: {checked}", flush=True)
    assert checked >= 100
