"""GPU parity of the on-device library simulation (tm_simulate_library)
against the oracle's kinematical simulation (Section 2.1), for the three
lattices of the workloads, and indexing with a simulated library. Runs only
on an MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

# (lattice, params, atoms, Laue sector) of the workloads' phases
PHASES = {
    "fcc": (np.eye(3) / 4.05, [[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]),
    "ortho": (np.diag([1 / 5.1, 1 / 7.3, 1 / 4.6]), [[0, 0, 0]]),
    "hcp": (np.linalg.inv(np.array([[2.95, 0, 0], [-1.475, 2.95 * np.sqrt(3) / 2, 0],
                                    [0, 0, 2.95 * 1.59]])).T, [[0, 0, 0], [1 / 3, 2 / 3, 0.5]]),
}
K = 1.0 / synth.wavelength_A(200.0)
S_MAX, G_MAX, G_LIM, REL_MIN = 0.05, 1.2, 1.4, 1e-3
MARGIN = 1e-9     # decisions closer than this to a threshold may go either way


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _orientations(rng, T):
    v = rng.standard_normal((T, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    e = np.stack([np.arccos(v[:, 2]), np.arctan2(v[:, 0], v[:, 1])], axis=1)
    e[0] = (0.0, 0.0)              # zone axis [001]: many equal intensities
    e[1] = (np.pi / 2, np.pi / 4)  # beam along [110]
    return e


def _borderline(g_c, F2, Phi, phi2, max_spots):
    """True if some decision of the oracle for this orientation lies within
    MARGIN of its threshold: relrod edge, projection radius, relative
    intensity floor, or two kept intensities (order and the max_spots cut)."""
    M = oracle.bunge_matrix64(0.0, Phi, phi2).T
    gs = g_c @ M.T
    s = oracle.excitation_error64(gs, K)
    shape = oracle.shape_factor64(s, S_MAX)
    r = np.hypot(gs[:, 0], gs[:, 1])
    if np.any(np.abs(np.abs(s) - S_MAX) < MARGIN) or np.any(np.abs(r - G_MAX) < MARGIN):
        return True
    ok = (shape > 0) & (r <= G_MAX)
    if not ok.any():
        return False
    I = F2 * shape
    top = I[ok].max()
    if np.any(np.abs(I[ok] - REL_MIN * top) < MARGIN * top):
        return True
    # equal or nearly equal intensities: their order rests on the last bits
    kept = np.sort(I[ok & (I >= REL_MIN * top)])[::-1]
    return bool(np.any(np.abs(np.diff(kept)) < MARGIN * top))


@pytest.mark.parametrize("phase", ["fcc", "ortho", "hcp"])
def test_simulation_equals_oracle(tm, phase):
    import torch
    Bm, atoms = PHASES[phase]
    atoms = np.array(atoms, dtype=float)
    f = np.ones(len(atoms))
    rng = np.random.default_rng(70 + len(phase))
    T, S = 160, 100
    e = _orientations(rng, T)
    _say("simulate", phase, T, "orientations, max_spots", S)
    kx, ky, I, cnt = tm.simulate_library(Bm, atoms, f, G_LIM, torch.from_numpy(e).cuda(), K,
                                         S_MAX, G_MAX, REL_MIN, S, csr=False)
    kx, ky, I, cnt = (a.cpu().numpy() for a in (kx, ky, I, cnt))
    _, g_c, F2 = oracle.reflections64(Bm, atoms, f, G_LIM)
    exact = border = 0
    for t in range(T):
        okx, oky, oI = oracle.simulate_template64(g_c, F2, e[t, 0], e[t, 1], K, S_MAX, G_MAX,
                                                  REL_MIN, S)
        n = int(cnt[t])
        same = (n == len(okx) and np.allclose(kx[t, :n], okx, atol=1e-12)
                and np.allclose(ky[t, :n], oky, atol=1e-12) and np.allclose(I[t, :n], oI, atol=1e-12))
        if same:
            exact += 1
            continue
        assert _borderline(g_c, F2, e[t, 0], e[t, 1], S), (phase, t, n, len(okx))
        border += 1
    _say(f"{phase}: {exact} identical, {border} borderline of {T}")
    assert exact >= T - 2


def test_simulated_library_indexes_like_the_generator_library(tm, c1, c1_lib):
    """The tiny workload's library simulated on the device (same crystal,
    orientations and parameters as the generator's) gives the same CSR
    arrays, and indexing with it gives the same matches."""
    import torch
    Bm, atoms = PHASES["fcc"]
    atoms = np.array(atoms, dtype=float)
    e = torch.from_numpy(synth.template_euler(c1)).cuda()
    _say("simulated c1 library vs generator library")
    sim = tm.simulate_library(Bm, atoms, np.ones(len(atoms)), c1.g_max + 0.2, e,
                              1.0 / synth.wavelength_A(c1.kv), c1.s_max, c1.g_max, 1e-3,
                              c1.phases[0].max_spots)
    assert np.array_equal(sim["offsets"], c1_lib["offsets"])
    for key in ("kx", "ky", "intensity"):
        assert np.allclose(sim[key], c1_lib[key], atol=1e-12)
    grid = tm.PolarGrid(R=c1.R, n_theta=c1.n_theta, cx=c1.cx, cy=c1.cy)
    px = synth.px_per_inv_A(c1)
    lib_a = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"], px, grid)
    lib_b = tm.Library(sim["kx"], sim["ky"], sim["intensity"], sim["offsets"], px, grid)
    x = torch.from_numpy(synth.make_patterns(c1, c1_lib, range(32))).cuda()
    polar, norms, _ = tm.polar_transform(x, grid)
    ra = [o.cpu().numpy() for o in tm.match_batch(lib_a, polar, norms, 5)]
    rb = [o.cpu().numpy() for o in tm.match_batch(lib_b, polar, norms, 5)]
    assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])
    assert np.allclose(ra[2], rb[2], atol=1e-6)


def test_simulation_edge_cases(tm):
    import torch
    Bm, atoms = PHASES["fcc"]
    atoms = np.array(atoms, dtype=float)
    f = np.ones(len(atoms))
    _say("simulate edge cases")
    e = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    kx, ky, I, cnt = tm.simulate_library(Bm, atoms, f, G_LIM, e, K, S_MAX, G_MAX, csr=False)
    assert cnt.numel() == 0
    # a relrod too thin for any reflection off the zero layer's curvature:
    # the [001] zone keeps only spots within s_max of the sphere
    e = torch.tensor([[0.0, 0.0], [0.9, 0.4]], dtype=torch.float64, device="cuda")
    kx, ky, I, cnt = tm.simulate_library(Bm, atoms, f, G_LIM, e, K, 1e-6, G_MAX, csr=False)
    _, g_c, F2 = oracle.reflections64(Bm, atoms, f, G_LIM)
    for t in range(2):
        okx, _, _ = oracle.simulate_template64(g_c, F2, float(e[t, 0]), float(e[t, 1]), K, 1e-6,
                                               G_MAX, REL_MIN, 100)
        assert int(cnt[t]) == len(okx)
    # max_spots = 1: the brightest spot only, intensity 1
    kx, ky, I, cnt = tm.simulate_library(Bm, atoms, f, G_LIM, e, K, S_MAX, G_MAX, max_spots=1,
                                         csr=False)
    assert cnt.cpu().tolist() == [1, 1] and np.allclose(I.cpu().numpy()[:, 0], 1.0)


def test_simulation_spills_past_the_lds_list(tm):
    """A relrod so wide that most reflections are excited: each wave's
    candidate list runs past its 256 LDS entries into the global spill
    area; results still equal the oracle's."""
    import torch
    Bm, atoms = PHASES["ortho"]
    atoms = np.array(atoms, dtype=float)
    f = np.ones(len(atoms))
    rng = np.random.default_rng(77)
    T, S, s_max = 24, 4096, 2.0
    e = _orientations(rng, T)
    _say("simulate with spills: ortho, s_max", s_max, T)
    kx, ky, I, cnt = tm.simulate_library(Bm, atoms, f, G_LIM, torch.from_numpy(e).cuda(), K,
                                         s_max, G_MAX, 0.0, S, csr=False)
    kx, ky, I, cnt = (a.cpu().numpy() for a in (kx, ky, I, cnt))
    _, g_c, F2 = oracle.reflections64(Bm, atoms, f, G_LIM)
    for t in range(T):
        okx, oky, oI = oracle.simulate_template64(g_c, F2, e[t, 0], e[t, 1], K, s_max, G_MAX,
                                                  0.0, S)
        n = int(cnt[t])
        assert n == len(okx) and n > 600, (t, n, len(okx))
        # many equal intensities: compare as sets of spots (distinct positions)
        go = np.lexsort((np.round(ky[t, :n], 6), np.round(kx[t, :n], 6)))
        wo = np.lexsort((np.round(oky, 6), np.round(okx, 6)))
        for a, b in ((kx[t, :n], okx), (ky[t, :n], oky), (I[t, :n], oI)):
            assert np.allclose(a[go], b[wo], atol=1e-12), t
        assert np.all(np.diff(I[t, :n]) <= 1e-12)
