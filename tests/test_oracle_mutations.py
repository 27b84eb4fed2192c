"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each case monkeypatches one oracle function with a plausible bug (a swapped
axis, a wrong sign, a dropped term, a wrong tie rule) and runs the pins that
should catch it."""
import numpy as np
import pytest

import oracle
import oracle.library as olibmod
import oracle.match as omatch
import oracle.orient as oorient
import oracle.polar as opolar
import oracle.prefilter as opre
import oracle.preprocess as oprep
import oracle.simulate as osim
import test_oracle_pins as pins


def _swapped_coords(R, n_theta, r0, dr, cx, cy):
    x, y = _orig_coords(R, n_theta, r0, dr, cx, cy)
    return cy + (x - cx), cx + (y - cy)          # x and y exchanged


_orig_coords = opolar.polar_coords64


def _clockwise_coords(R, n_theta, r0, dr, cx, cy):
    x, y = _orig_coords(R, n_theta, r0, dr, cx, cy)
    return x, 2 * cy - y                         # angle measured the other way


def _bilinear_transposed(img, x, y):
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = x - x0, y - y0
    xi, yi = x0.astype(np.int64), y0.astype(np.int64)
    p = opolar._pixel
    return ((1 - fx) * (1 - fy) * p(img, yi, xi) + fy * (1 - fx) * p(img, yi, xi + 1)
            + (1 - fy) * fx * p(img, yi + 1, xi) + fx * fy * p(img, yi + 1, xi + 1))


_orig_num = omatch._numerators


def _num_wrong_sign(P, lib, t_lo, t_hi):
    # slides the template the other way: P[j, k - s]
    return _orig_num(P[:, ::-1][:, np.r_[len(P[0]) - 1, 0:len(P[0]) - 1]], lib, t_lo, t_hi)


def _num_no_wrap(P, lib, t_lo, t_hi):
    Pz = np.concatenate([P, np.zeros_like(P)], axis=1)
    n = P.shape[1]
    a, b = lib.starts[t_lo], lib.starts[t_hi]
    out = np.zeros((t_hi - t_lo, n))
    s = np.arange(n)
    g = Pz[lib.J[a:b, None], lib.K[a:b, None] + s[None, :]] * lib.Wt[a:b, None]
    np.add.at(out, lib.tid[a:b] - t_lo, g)
    return out


_orig_tp = olibmod.template_pixels64


def _tp_mirror_not_reflected(kx, ky, intensity, offsets, px_per, R, n_theta, r0=0.0, dr=1.0,
                             mirror=True, unit=False, keep_direct_beam=False):
    base = _orig_tp(kx, ky, intensity, offsets, px_per, R, n_theta, r0, dr, False, unit,
                    keep_direct_beam)
    return base + base if mirror else base


def _tp_no_merge(kx, ky, intensity, offsets, px_per, R, n_theta, r0=0.0, dr=1.0,
                 mirror=True, unit=False, keep_direct_beam=False):
    out = []
    offsets = np.asarray(offsets)
    for sign in ((1.0, -1.0) if mirror else (1.0,)):
        for t in range(len(offsets) - 1):
            a, b = offsets[t], offsets[t + 1]
            x, y = np.asarray(kx[a:b]), sign * np.asarray(ky[a:b])
            w = np.ones(b - a) if unit else np.asarray(intensity[a:b], dtype=float)
            keep = ~((x == 0) & (y == 0)) | keep_direct_beam
            j = np.rint((px_per * np.hypot(x, y) - r0) / dr)
            k = np.mod(np.rint(np.arctan2(y, x) * n_theta / (2 * np.pi)), n_theta)
            keep &= (j >= 0) & (j < R)
            out.append((j[keep].astype(int), k[keep].astype(int), w[keep]))   # duplicates kept apart
    return out


def _match_last_max(P, lib, pnorm=None, chunk=512):
    Q = oracle.scores64(P, lib, pnorm)
    n = Q.shape[1]
    arg = n - 1 - np.argmax(Q[:, ::-1], axis=1)
    return Q[np.arange(len(Q)), arg], arg


def _topn_ties_high_index(best, arg, N, templates=None):
    tids = np.arange(len(best)) if templates is None else np.asarray(templates)
    order = np.lexsort((-tids, -np.asarray(best)))[:N]
    return tids[order], np.asarray(arg)[order], np.asarray(best)[order]


_orig_bunge = oorient.bunge_matrix64


def _bunge_transposed(phi1, Phi, phi2):
    return _orig_bunge(phi1, Phi, phi2).T        # active and passive confused


def _mirror_about_y(Phi, phi2, phi, mirrored):
    M = oorient.bunge_matrix64(0.0, Phi, phi2).T
    if mirrored:
        M = np.diag([-1.0, 1.0, -1.0]) @ M       # pi about sample y: spots (-kx, ky)
    M = oorient.rot_z_active64(phi) @ M
    return oorient.euler_from_matrix64(M.T)


def _sector_xy_swapped(v, laue):
    w = _orig_sector(v, laue)
    return np.array([w[1], w[0], w[2]]) if laue == "m-3m" else w


_orig_sector = oorient.sector_direction64


def _ipf_unreduced(euler_a, euler_b, laue):
    ga, gb = oorient.bunge_matrix64(*euler_a), oorient.bunge_matrix64(*euler_b)
    return np.abs(np.arccos(np.clip(np.sum(ga * gb, axis=0), -1.0, 1.0)))


def _ewald_wrong_side(g_sample, k):
    d = g_sample + np.array([0.0, 0.0, k])     # sphere centred at (0, 0, -k)
    return k - np.sqrt(np.sum(d * d, axis=-1))


def _make_sim(transpose=True, ties_reversed=False):
    def sim(g_c, F2, Phi, phi2, k, s_max, g_max, rel_min, max_spots):
        M = oorient.bunge_matrix64(0.0, Phi, phi2)
        M = M.T if transpose else M
        gs = np.asarray(g_c) @ M.T
        shape = osim.shape_factor64(osim.excitation_error64(gs, k), s_max)
        I = np.asarray(F2) * shape
        idx = np.nonzero((shape > 0) & (np.hypot(gs[:, 0], gs[:, 1]) <= g_max))[0]
        top = I[idx].max()
        idx = idx[I[idx] >= rel_min * top]
        key = (lambda i: (-I[i], -i)) if ties_reversed else (lambda i: (-I[i], i))
        order = np.array(sorted(idx.tolist(), key=key)[:max_spots], dtype=np.int64)
        return gs[order, 0], gs[order, 1], I[order] / top
    return sim


_orig_convolve = oprep.convolve_axis64


def _convolve_zero_border(img, w, axis):
    r = (len(w) - 1) // 2
    pad = [(0, 0), (0, 0)]
    pad[axis] = (r, r)
    p = np.pad(np.asarray(img, dtype=np.float64), pad)
    n = np.asarray(img).shape[axis]
    return sum(w[t] * np.take(p, np.arange(n) + t, axis=axis) for t in range(2 * r + 1))


def _shift_wrong_way(img, dx, dy):
    return _orig_shift(img, -dx, -dy)


_orig_shift = oprep.shift_image64



def _nearest_floor(img, x, y):
    return opolar._pixel(img, np.floor(y).astype(np.int64), np.floor(x).astype(np.int64))


def _nearest_swapped(img, x, y):
    return opolar._pixel(img, np.rint(x).astype(np.int64), np.rint(y).astype(np.int64))


def _nearest_half_up(img, x, y):
    return opolar._pixel(img, np.floor(y + 0.5).astype(np.int64),
                         np.floor(x + 0.5).astype(np.int64))


def _prefilter_unnormalised(prof_P, prof_T, keep):
    import math
    dots = prof_T @ np.asarray(prof_P, dtype=np.float64)
    n_keep = min(len(prof_T), int(math.ceil(keep * len(prof_T))))
    return np.lexsort((np.arange(len(prof_T)), -dots))[:n_keep].astype(np.int64), dots


def _profile_wrong_axis(P):
    return np.asarray(P, dtype=np.float64).sum(axis=0)


_orig_prefilter = opre.prefilter64


def _prefilter_ties_high(prof_P, prof_T, keep):
    kept, cos = _orig_prefilter(prof_P, prof_T, keep)
    import math
    n_keep = len(kept)
    order = np.lexsort((-np.arange(len(prof_T)), -cos))[:n_keep]
    return order.astype(np.int64), cos


def _prefilter_floor_count(prof_P, prof_T, keep):
    kept, cos = _orig_prefilter(prof_P, prof_T, 1.0)
    return kept[:max(1, int(keep * len(prof_T)))], cos


CASES = [
    ("x/y swapped in polar coordinates", opolar, "polar_coords64", _swapped_coords,
     [pins.test_p9_polar_reproduces_bilinear_functions]),
    ("angle measured clockwise", opolar, "polar_coords64", _clockwise_coords,
     [pins.test_p9_polar_reproduces_bilinear_functions, pins.test_p6_polar_equals_scipy_map_coordinates]),
    ("bilinear weights transposed", opolar, "bilinear64", _bilinear_transposed,
     [pins.test_p6_polar_equals_scipy_map_coordinates]),
    ("template slid the wrong way", omatch, "_numerators", _num_wrong_sign,
     [pins.test_p2_cartesian_rotated_template_equals_polar_shift, pins.test_p3_roll_by_one_bin]),
    ("no wraparound", omatch, "_numerators", _num_no_wrap,
     [pins.test_p6_numerator_equals_fft_cross_correlation]),
    ("mirror not reflected", olibmod, "template_pixels64", _tp_mirror_not_reflected,
     [pins.test_p11_mirror_identity]),
    ("duplicate spots not merged", olibmod, "template_pixels64", _tp_no_merge,
     [pins.test_template_pixels_rounding_merge_and_drop]),
    ("last maximum instead of first", omatch, "match_exact64", _match_last_max,
     [pins.test_p7_topn_brute_force]),
    ("ties ranked by higher index", omatch, "topn64", _topn_ties_high_index,
     [pins.test_p7_topn_brute_force]),
    ("Bunge matrix transposed", oorient, "bunge_matrix64", _bunge_transposed,
     [pins.test_bunge_matrix_equals_scipy_intrinsic_zxz]),
    ("mirror read as a rotation about y", oorient, "match_orientation64", _mirror_about_y,
     [pins.test_match_orientation_reproduces_rotated_and_mirrored_spots]),
    ("cubic sector with x and y swapped", oorient, "sector_direction64", _sector_xy_swapped,
     [lambda: pins.test_laue_group_is_a_group_and_sector_is_fundamental("m-3m", 48)]),
    ("Eq. (2) without the symmetry reduction", oorient, "ipf_deviation64", _ipf_unreduced,
     [pins.test_eq2_closed_forms]),
    ("Ewald sphere on the wrong side", osim, "excitation_error64", _ewald_wrong_side,
     [pins.test_excitation_error_ewald_geometry]),
    ("orientation applied untransposed", osim, "simulate_template64", _make_sim(False),
     [pins.test_phi2_rotates_a_zone_pattern_in_plane]),
    ("equal intensities in reverse grid order", osim, "simulate_template64",
     _make_sim(True, True), [pins.test_fcc_001_zone_axis_pattern]),
    ("Gaussian with a zero border", oprep, "convolve_axis64", _convolve_zero_border,
     [lambda: pins.test_gaussian_equals_scipy_reflect(2.5)]),
    ("centring shift the wrong way", oprep, "shift_image64", _shift_wrong_way,
     [pins.test_shift_integer_fraction_and_round_trip, pins.test_preprocess_centres_an_offset_beam]),
    ("nearest sample by floor instead of rint", opolar, "nearest64", _nearest_floor,
     [pins.test_nearest_on_pixel_centres_fixes_axes, pins.test_nearest_equals_brute_force_closest_centre]),
    ("nearest sample with x and y swapped", opolar, "nearest64", _nearest_swapped,
     [pins.test_nearest_on_pixel_centres_fixes_axes]),
    ("nearest half-pixel ties rounded up", opolar, "nearest64", _nearest_half_up,
     [pins.test_nearest_half_pixel_ties_round_half_to_even]),
    ("pre-filter by unnormalised dot product", opre, "prefilter64", _prefilter_unnormalised,
     [pins.test_prefilter_own_image_has_cosine_one_and_ranks_first,
      pins.test_prefilter_cosine_equals_half_squared_distance_of_unit_profiles]),
    ("image profile summed over radii", opolar, "profile64", _profile_wrong_axis,
     [pins.test_prefilter_own_image_has_cosine_one_and_ranks_first]),
    ("pre-filter ties to the higher index", opre, "prefilter64", _prefilter_ties_high,
     [pins.test_prefilter_own_image_has_cosine_one_and_ranks_first]),
    ("pre-filter keeps floor(f T)", opre, "prefilter64", _prefilter_floor_count,
     [pins.test_prefilter_invariances_and_count]),
]


@pytest.mark.parametrize("name,mod,attr,bad,tests", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, name, mod, attr, bad, tests):
    monkeypatch.setattr(mod, attr, bad)
    # functions re-exported at package level or imported into sibling modules
    for m in (oracle, omatch, pins.oracle):
        if hasattr(m, attr):
            monkeypatch.setattr(m, attr, bad)
    import oracle.prefilter as opre
    if hasattr(opre, attr):
        monkeypatch.setattr(opre, attr, bad)
    caught = 0
    for t in tests:
        try:
            t()
        except AssertionError:
            caught += 1
    assert caught >= 1, f"planted mistake '{name}' passed every pin"
