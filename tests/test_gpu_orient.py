"""GPU parity of the orientation output (tm_orientations) and of Eq. (2)
(tm_ipf_deviation) against the oracle, and the physical accuracy of indexed
synthetic patterns against the generator's ground truth. Runs only on an
MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * np.pi


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _lib_euler(rng, T):
    e = np.stack([np.arccos(rng.uniform(-1, 1, T)), rng.uniform(0, TWO_PI, T)], axis=1)
    e[0] = (0.0, 1.3)          # beam along crystal z: Phi = 0
    e[1] = (np.pi, 4.2)        # Phi = pi
    return e


def _same_rotation(e_gpu, e_ref):
    return np.allclose(oracle.bunge_matrix64(*e_gpu), oracle.bunge_matrix64(*e_ref), atol=1e-12)


@pytest.mark.parametrize("refined", [False, True])
def test_orientations_equal_oracle(tm, refined):
    import torch
    rng = np.random.default_rng(50)
    T, B, N, n_theta = 40, 96, 4, 360
    le = _lib_euler(rng, T)
    tt = rng.integers(0, 2 * T, (B, N)).astype(np.int32)
    tt[0, 0], tt[1, 1], tt[2, 2] = -1, 2 * T, 2 * T + 5          # not a template: NaN
    tt[3, :2] = (0, T)                                           # Phi = 0, and its mirror
    tt[4, :2] = (1, T + 1)                                       # Phi = pi, and its mirror
    bins = rng.integers(0, n_theta, (B, N)).astype(np.int32)
    deg = rng.uniform(-0.5, 360.0, (B, N)).astype(np.float32)
    _say("orientations", "refined" if refined else "bins", B, N, T)
    dev = torch.device("cuda")
    out = tm.orientations(torch.from_numpy(le).to(dev), torch.from_numpy(tt).to(dev),
                          top_angle=None if refined else torch.from_numpy(bins).to(dev),
                          angle_deg=torch.from_numpy(deg).to(dev) if refined else None,
                          n_theta=n_theta).cpu().numpy()
    for b in range(B):
        for n in range(N):
            t = int(tt[b, n])
            if t < 0 or t >= 2 * T:
                assert np.all(np.isnan(out[b, n])), (b, n)
                continue
            phi = np.radians(float(deg[b, n])) if refined else bins[b, n] * TWO_PI / n_theta
            ref = oracle.match_orientation64(le[t % T, 0], le[t % T, 1], phi, t >= T)
            got = out[b, n]
            assert _same_rotation(got, ref), (b, n, got, ref)
            assert 0.0 <= got[0] < TWO_PI and 0.0 <= got[1] <= np.pi and 0.0 <= got[2] < TWO_PI
            if np.sin(ref[1]) > 1e-6:
                d = (got - ref + np.pi) % TWO_PI - np.pi
                assert np.allclose(d, 0.0, atol=1e-11), (b, n, got, ref)
            else:
                assert got[2] == 0.0 and abs(got[1] - ref[1]) < 1e-12


@pytest.mark.parametrize("laue", ["m-3m", "mmm", "6/mmm"])
def test_ipf_deviation_equals_oracle(tm, laue):
    import torch
    rng = np.random.default_rng(51 + len(laue))
    B, N = 160, 3
    ea = np.stack([rng.uniform(0, TWO_PI, (B, N)), np.arccos(rng.uniform(-1, 1, (B, N))),
                   rng.uniform(0, TWO_PI, (B, N))], axis=2)
    eb = np.stack([rng.uniform(0, TWO_PI, B), np.arccos(rng.uniform(-1, 1, B)),
                   rng.uniform(0, TWO_PI, B)], axis=1)
    # symmetry-equivalent pairs (deviation 0) and small rotations
    ops = [o for o in oracle.symmetry_operators64(laue) if np.linalg.det(o) > 0]
    for b in range(0, 40):
        S = ops[rng.integers(len(ops))]
        eb[b] = oracle.euler_from_matrix64(S @ oracle.bunge_matrix64(*ea[b, 0]))
    for b in range(40, 60):
        eb[b] = ea[b, 0] + rng.normal(0, 0.01, 3)
        eb[b, 1] = abs(eb[b, 1])
    _say("ipf deviation", laue, B)
    dev = torch.device("cuda")
    got = tm.ipf_deviation(torch.from_numpy(ea).to(dev), torch.from_numpy(eb).to(dev),
                           laue).cpu().numpy()
    for b in range(B):
        want = oracle.ipf_deviation64(ea[b, 0], eb[b], laue)
        assert np.allclose(got[b], want, atol=1e-7), (b, got[b], want)
    assert np.all(got[:40] < 1e-6)


def test_indexed_orientations_match_ground_truth(tm, c1, c1_lib):
    """Patterns rendered from library templates at random in-plane angles
    (and mirrored at random): where the best match is the generating
    template, its orientation reproduces the ground truth up to the angular
    bin (1 degree: IPF-z exact, IPF-x/y within half a bin), and the sub-bin
    angles bring it closer."""
    import torch
    B = 64
    _say("accuracy vs ground truth, c1", B)
    grid = tm.PolarGrid(R=c1.R, n_theta=c1.n_theta, cx=c1.cx, cy=c1.cy)
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                     synth.px_per_inv_A(c1), grid)
    T = lib.n_total // 2
    x = torch.from_numpy(synth.make_patterns(c1, c1_lib, range(B))).cuda()
    polar, norms, _ = tm.polar_transform(x, grid)
    tt, ts, _ = tm.match_batch(lib, polar, norms, 1)
    deg = tm.refine_angles(lib, polar, norms, tt, ts)
    le = torch.from_numpy(synth.template_euler(c1)).cuda()
    truth = [synth.ground_truth(c1, i, T) for i in range(B)]
    t_true = torch.tensor([[t + (T if m else 0)] for t, m, _ in truth], dtype=torch.int32).cuda()
    a_true = torch.tensor([[np.degrees(p)] for _, _, p in truth], dtype=torch.float32).cuda()
    e_true = tm.orientations(le, t_true, angle_deg=a_true, n_theta=c1.n_theta)
    e_bin = tm.orientations(le, tt, top_angle=ts, n_theta=c1.n_theta)
    e_ref = tm.orientations(le, tt, angle_deg=deg, n_theta=c1.n_theta)
    d_bin = np.degrees(tm.ipf_deviation(e_bin, e_true, "m-3m").cpu().numpy())
    d_ref = np.degrees(tm.ipf_deviation(e_ref, e_true, "m-3m").cpu().numpy())
    hit = tt.cpu().numpy()[:, 0] == t_true.cpu().numpy()[:, 0]
    _say(f"generating template found for {hit.sum()} of {B}; median IPF-x dev "
         f"bins {np.median(d_bin[hit, 0]):.3f} deg, refined {np.median(d_ref[hit, 0]):.3f} deg")
    assert hit.sum() >= B // 2
    assert np.all(d_bin[hit, 2] < 1e-5)
    # the best bin is the nearest one, or (with noise) its neighbour
    assert np.all(d_bin[hit, :2] <= 1.5 + 1e-3)
    assert np.median(d_bin[hit, :2]) <= 0.5
    assert np.median(d_ref[hit, :2]) < np.median(d_bin[hit, :2])
