"""GPU parity of the preprocessing steps (tm_preprocess: direct-beam
centring, difference of Gaussians, blur, threshold; Section 4.1) against the
oracle, and indexing of off-centre patterns after centring. Runs only on an
MI355X (marked gpu)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth

pytestmark = pytest.mark.gpu

OPTS = {
    "all": dict(r_box=8, frac=0.5, sigma_min=1.0, sigma_max=6.0, sigma_blur=1.0, threshold=0.0),
    "no_centring": dict(r_box=-1, frac=0.5, sigma_min=0.7, sigma_max=3.0, sigma_blur=1.5,
                        threshold=0.001),
    "no_dog": dict(r_box=6, frac=0.3, sigma_min=0.0, sigma_max=0.0, sigma_blur=2.0,
                   threshold=float("-inf")),
    "centre_only": dict(r_box=8, frac=0.2, sigma_min=0.0, sigma_max=0.0, sigma_blur=0.0,
                        threshold=float("-inf")),
}


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2111_07347_amd as tm
    return tm


def _offset_patterns(cfg, lib, n, seed, max_shift=3.0):
    """Generated patterns moved by random sub-pixel offsets (the direct beam
    then sits off the centre), float64 and the offsets."""
    rng = np.random.default_rng(seed)
    imgs = synth.make_patterns(cfg, lib, range(n)).astype(np.float64)
    d = rng.uniform(-max_shift, max_shift, (n, 2))
    out = np.stack([ndimage.shift(imgs[i], (d[i, 1], d[i, 0]), order=1, mode="constant")
                    for i in range(n)])
    return out, d


def _compare(got, want, pre, threshold, tag):
    scale = max(1.0, float(np.abs(pre).max()))
    tol = 2e-5 * scale
    near = np.abs(pre - threshold) <= 4 * tol if np.isfinite(threshold) else np.zeros_like(pre, bool)
    bad = (np.abs(got - want) > tol) & ~near
    assert not bad.any(), (tag, int(bad.sum()), float(np.abs(got - want)[bad].max()))


@pytest.mark.parametrize("name", sorted(OPTS))
@pytest.mark.parametrize("dtype", ["f32", "u16"])
def test_preprocess_equals_oracle(tm, c1, c1_lib, name, dtype):
    import torch
    o = OPTS[name]
    imgs, _ = _offset_patterns(c1, c1_lib, 6, 90)
    if dtype == "u16":
        imgs = np.clip(np.rint(imgs * 1000), 0, 65535)
        x = torch.from_numpy(imgs.astype(np.uint16).view(np.int16)).cuda()
    else:
        x = torch.from_numpy(imgs.astype(np.float32)).cuda()
        imgs = imgs.astype(np.float32).astype(np.float64)
    _say("preprocess", name, dtype, imgs.shape)
    out, cen = tm.preprocess(x, **o)
    out, cen = out.cpu().numpy(), cen.cpu().numpy()
    for b in range(len(imgs)):
        want, (cx, cy) = oracle.preprocess64(imgs[b], **o)
        pre, _ = oracle.preprocess64(imgs[b], **{**o, "threshold": float("-inf")})
        assert abs(cen[b, 0] - cx) < 1e-9 and abs(cen[b, 1] - cy) < 1e-9, (b, cen[b], cx, cy)
        _compare(out[b], want, pre, o["threshold"], (name, dtype, b))


@pytest.mark.parametrize("shape", [(100, 90), (7, 5), (1, 33)])
def test_preprocess_ragged_and_tiny_images(tm, shape):
    """Sizes not multiple of anything, and images narrower than the
    Gaussian's radius (the mirror folds several times)."""
    import torch
    rng = np.random.default_rng(91)
    imgs = rng.random((3,) + shape).astype(np.float32)
    o = dict(r_box=2, frac=0.4, sigma_min=1.0, sigma_max=6.0, sigma_blur=1.0, threshold=0.0)
    _say("preprocess ragged", shape)
    out, cen = tm.preprocess(torch.from_numpy(imgs).cuda(), **o)
    out, cen = out.cpu().numpy(), cen.cpu().numpy()
    for b in range(3):
        want, (cx, cy) = oracle.preprocess64(imgs[b].astype(np.float64), **o)
        pre, _ = oracle.preprocess64(imgs[b].astype(np.float64), **{**o, "threshold": float("-inf")})
        assert abs(cen[b, 0] - cx) < 1e-9 and abs(cen[b, 1] - cy) < 1e-9
        _compare(out[b], want, pre, 0.0, (shape, b))


@pytest.mark.parametrize("shape,sigmas", [((300, 260), (2.0, 15.9, 3.3)), ((64, 516), (1.0, 6.0, 1.0))])
def test_preprocess_wide_tall_images_and_largest_radius(tm, shape, sigmas):
    """Rows wider than one 256-column chunk (the row pass walks several),
    images taller than the column-strip tile (the per-column pass), and the
    largest supported radius (sigma 15.9: 64 taps each side)."""
    import torch
    rng = np.random.default_rng(93)
    imgs = (rng.random((2,) + shape) * 3.0).astype(np.float32)
    o = dict(r_box=5, frac=0.4, sigma_min=sigmas[0], sigma_max=sigmas[1], sigma_blur=sigmas[2],
             threshold=0.05)
    _say("preprocess wide/tall", shape, sigmas)
    out, cen = tm.preprocess(torch.from_numpy(imgs).cuda(), **o)
    out, cen = out.cpu().numpy(), cen.cpu().numpy()
    for b in range(2):
        want, (cx, cy) = oracle.preprocess64(imgs[b].astype(np.float64), **o)
        pre, _ = oracle.preprocess64(imgs[b].astype(np.float64), **{**o, "threshold": float("-inf")})
        assert abs(cen[b, 0] - cx) < 1e-9 and abs(cen[b, 1] - cy) < 1e-9
        _compare(out[b], want, pre, 0.05, (shape, b))


def test_preprocess_degenerate_inputs(tm):
    import torch
    _say("preprocess degenerate")
    z = torch.zeros((2, 16, 16), dtype=torch.float32, device="cuda")
    out, cen = tm.preprocess(z)
    assert torch.all(out == 0) and np.allclose(cen.cpu().numpy(), 8.0)
    e = torch.zeros((0, 16, 16), dtype=torch.float32, device="cuda")
    out, cen = tm.preprocess(e)
    assert out.shape == (0, 16, 16)


def test_centring_restores_indexing_of_offset_patterns(tm, c1, c1_lib):
    """Patterns moved off the centre by up to 3 px: indexed as they are, the
    polar transform about the image centre misses the beam; after centring
    the top-1 agrees with that of the unmoved patterns."""
    import torch
    B = 32
    imgs, _ = _offset_patterns(c1, c1_lib, B, 92)
    ref = synth.make_patterns(c1, c1_lib, range(B))
    grid = tm.PolarGrid(R=c1.R, n_theta=c1.n_theta, cx=c1.cx, cy=c1.cy)
    lib = tm.Library(c1_lib["kx"], c1_lib["ky"], c1_lib["intensity"], c1_lib["offsets"],
                     synth.px_per_inv_A(c1), grid)
    _say("centring then indexing", B)

    def top1(x):
        polar, norms, _ = tm.polar_transform(x, grid)
        return tm.match_batch(lib, polar, norms, 1)[0].cpu().numpy()[:, 0]
    t_ref = top1(torch.from_numpy(ref).cuda())
    x = torch.from_numpy(imgs.astype(np.float32)).cuda()
    t_off = top1(x)
    c, _ = tm.preprocess(x, r_box=8, frac=0.2, sigma_min=0.0, sigma_max=0.0, sigma_blur=0.0,
                         threshold=float("-inf"))
    t_cen = top1(c)
    a_off, a_cen = np.mean(t_off == t_ref), np.mean(t_cen == t_ref)
    _say(f"top-1 as the unmoved patterns: off-centre {a_off:.2f}, centred {a_cen:.2f}")
    assert a_cen >= 0.8 and a_cen > a_off
