"""CPU checks of the mathematics behind the window upper bounds (no GPU).

The bound kernel bounds C(s) = sum_i w_i P[j_i, (k_i + s) mod n] over the
window of win = ceil(n / 4) shifts starting at S win by

    U_S = sum_i w_i M[j_i, (k_i + S win - e_iS) mod n],
    M[j, x] = max(0, max_{0 <= d < wlen} P[j, (x + d) mod n]),

with dl = 4 win - n, wlen = min(win + dl, n) and e_iS = dl when
floor(k_i / win) + S >= 4 (else 0). It stores a pixel's four maxima as the
dwords (M[r], M[r + 2 win]) and (M[r + win], M[r + 3 win]) at r = k mod win,
accumulates acc[i] += w M[r + i win] per quarter q = k // win, and rotates
the accumulators by one between quarters taken in cyclic order. These tests
check, on random data and widths with and without 4 | n, that U_S bounds
every shift of its window (so max_S U_S bounds the template's best score)
and that the rotated accumulation gives exactly the four U_S."""
import numpy as np
import pytest


def _window_max(P, wlen):
    n = P.shape[1]
    M = np.max(np.stack([np.roll(P, -d, axis=1) for d in range(wlen)]), axis=0)
    return np.maximum(M, 0.0)


def _u(M, j, k, w, n, win):
    dl = 4 * win - n
    return np.array([(w * M[j, (k + S * win - dl * ((k // win) + S >= 4)) % n]).sum()
                     for S in range(4)])


@pytest.mark.parametrize("n", [16, 17, 18, 19, 64, 90, 181, 360, 361, 720, 768])
def test_window_sums_bound_every_shift(n):
    rng = np.random.default_rng(n)
    win = -(-n // 4)
    wlen = min(5 * win - n, n)
    for _ in range(40):
        P = rng.standard_normal((3, n))
        M = _window_max(P, wlen)
        npx = int(rng.integers(1, 12))
        j = rng.integers(0, 3, npx)
        k = rng.integers(0, n, npx)
        w = rng.random(npx)
        U = _u(M, j, k, w, n, win)
        for S in range(4):
            for s in range(S * win, min(n, S * win + win)):
                assert U[S] >= (w * P[j, (k + s) % n]).sum() - 1e-12
        # every shift lies in one of the four windows
        assert 4 * win >= n


@pytest.mark.parametrize("n", [16, 19, 90, 181, 360, 361, 768])
def test_rotated_quarter_accumulation_equals_window_sums(n):
    rng = np.random.default_rng(1000 + n)
    win = -(-n // 4)
    wlen = min(5 * win - n, n)
    for _ in range(40):
        P = rng.standard_normal((3, n))
        M = _window_max(P, wlen)
        # the image: Y[j, c] = (M[c], M[c + 2 win]) for c < 2 win (mod n)
        Y = np.stack([M[:, np.arange(2 * win) % n], M[:, (np.arange(2 * win) + 2 * win) % n]],
                     axis=2)
        npx = int(rng.integers(1, 12))
        j = rng.integers(0, 3, npx)
        k = rng.integers(0, n, npx)
        w = rng.random(npx)
        quarters = [[] for _ in range(4)]
        for jj, kk, ww in zip(j, k, w):
            quarters[kk // win].append((jj, kk % win, ww))
        start = int(rng.integers(0, 4))          # the lane's first quarter
        acc = np.zeros(4)
        for p in range(4):
            if p:
                acc = acc[[3, 0, 1, 2]]          # shift S moves from acc[S+q] to acc[S+q+1]
            for jj, r, ww in quarters[(start + p) % 4]:
                acc[0] += ww * Y[jj, r, 0]
                acc[2] += ww * Y[jj, r, 1]
                acc[1] += ww * Y[jj, r + win, 0]
                acc[3] += ww * Y[jj, r + win, 1]
        U = _u(M, j, k, w, n, win)
        # after the last quarter acc[i] holds shift (i - start - 3) mod 4
        q_last = (start + 3) % 4
        assert np.allclose([acc[(S + q_last) % 4] for S in range(4)], U, rtol=0, atol=1e-12)


def test_rounding_up_commutes_with_the_window_maximum():
    """The kernel rounds values up to float16 before taking window maxima:
    rounding up is monotone, so the maximum of rounded values is the rounded
    maximum."""
    rng = np.random.default_rng(5)
    x = rng.random(4000).astype(np.float32) * 1000.0

    def up16(v):
        h = v.astype(np.float16)
        h = np.where(h.astype(np.float32) < v, np.nextafter(h, np.float16(np.inf)), h)
        return h

    for _ in range(200):
        a, b = sorted(rng.integers(0, len(x), 2))
        if a == b:
            continue
        seg = x[a:b]
        assert up16(seg).max() == up16(np.array([seg.max()]))[0]
