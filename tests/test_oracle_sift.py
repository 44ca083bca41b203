"""Pins of the dereddening and sifting oracles (hand-built inputs, brute force,
library interpolation, statistics of white and red noise)."""
import math

import numpy as np
import pytest

import oracle as O

CAND = np.dtype([("series", "<i4"), ("harm", "<i4"), ("r_idx", "<i8"), ("z_idx", "<i4"), ("power", "<f4"),
                 ("sigma", "<f8"), ("r_fund", "<f8"), ("z_fund", "<f8"), ("f_hz", "<f8"), ("fdot_hz_s", "<f8")],
                align=True)


def test_blocks_cover_the_band_by_the_width_rule():
    for half in (2, 7, 1000, 65536):
        bl = O.deredden_blocks(half)
        assert bl[0][0] == 1 and bl[-1][1] == half
        for (b, e), (b2, _) in zip(bl, bl[1:]):
            assert e == b2 and e - b == min(200, 6 + b // 30)
        b, e = bl[-1]
        assert 1 <= e - b <= min(200, 6 + b // 30)


def test_constant_power_normalises_to_ln2():
    A = np.full(4097, 3.0 + 4.0j)
    Ah, m = O.deredden(A)
    assert np.allclose(m[1:4096], 25.0 / math.log(2.0), rtol=1e-14)
    assert np.allclose(np.abs(Ah[1:4096]) ** 2, math.log(2.0), rtol=1e-13)
    assert Ah[0] == 0 and Ah[4096] == 0


def test_piecewise_constant_blocks_interpolate_linearly():
    half = 3000
    bl = O.deredden_blocks(half)
    rng = np.random.default_rng(1)
    level = rng.uniform(1.0, 50.0, len(bl))
    A = np.zeros(half + 1, np.complex128)
    for (b, e), L in zip(bl, level):
        A[b:e] = math.sqrt(L)
    _, m = O.deredden(A)
    cen = np.array([(b + e - 1) / 2 for b, e in bl])
    k = np.arange(1, half)
    ref = np.interp(k, cen, level / math.log(2.0))       # constant beyond the end centres
    assert np.allclose(m[1:half], ref, rtol=1e-12)


def test_white_noise_stays_unit_mean():
    rng = np.random.default_rng(2)
    A = np.fft.rfft(rng.standard_normal(1 << 16))
    Ah, _ = O.deredden(A)
    p = np.abs(Ah[1:-1]) ** 2
    assert abs(p.mean() - 1.0) < 0.03


def test_red_noise_is_flattened():
    rng = np.random.default_rng(3)
    half = 1 << 15
    k = np.arange(half + 1, dtype=np.float64)
    k[0] = 1.0
    A = (rng.standard_normal(half + 1) + 1j * rng.standard_normal(half + 1)) * (1e4 / k)   # power ~ k^-2
    Ah, _ = O.deredden(A)
    p = np.abs(Ah) ** 2
    lo, hi = p[10:2000].mean(), p[20000:30000].mean()
    assert abs(lo - 1.0) < 0.1 and abs(hi - 1.0) < 0.05
    raw = np.abs(A) ** 2
    assert raw[10:2000].mean() / raw[20000:30000].mean() > 1e3


def _cands(rows):
    """rows: (series, harm, r_idx, sigma, f_hz); T = 50 s so r_fund = f T."""
    c = np.zeros(len(rows), CAND)
    for i, (s, h, r, sig, f) in enumerate(rows):
        c[i]["series"], c[i]["harm"], c[i]["r_idx"], c[i]["sigma"], c[i]["f_hz"] = s, h, r, sig, f
        c[i]["r_fund"] = f * 50.0
    return c


def test_duplicates_join_the_strongest_neighbour():
    T = 50.0
    f = 10.0
    c = _cands([(0, 1, 1, 8.0, f + 0.5 / T), (0, 1, 2, 10.0, f), (0, 1, 3, 9.0, f + 5.0 / T),
                (0, 1, 4, 7.0, f + 1.05 / T)])
    out = O.sift(c, tol_bins=1.1)
    assert [(i, h) for i, h, _, _ in out] == [(1, 3), (2, 1)]


def test_harmonics_of_stronger_survivors_are_dropped():
    T = 50.0
    f = 7.3
    c = _cands([(0, 1, 1, 12.0, f), (0, 2, 2, 9.0, 2 * f + 0.3 / T), (0, 4, 3, 8.0, 1.5 * f),
                (0, 1, 4, 7.5, f / 3 - 0.2 / T), (0, 1, 5, 7.0, 4 * f), (0, 1, 6, 6.5, 17 * f),
                (0, 1, 7, 6.0, 2 * f + 3.0 / T)])
    kept = [i for i, _, _, _ in O.sift(c, tol_bins=1.1, max_ratio=16)]
    # 2f, f/3 and 4f go; 3f/2 is no integer ratio, 17f is beyond 16, and 2f + 3/T is
    # 3 bins (> 2 x 1.1) from the second harmonic
    assert kept == [0, 2, 5, 6]
    assert [i for i, _, _, _ in O.sift(c, tol_bins=1.1, max_ratio=1)] == [0, 1, 2, 3, 4, 5, 6]
    # a weaker candidate never removes a stronger one
    c2 = _cands([(0, 1, 1, 5.0, f), (0, 1, 2, 9.0, 2 * f)])
    assert [i for i, _, _, _ in O.sift(c2)] == [1]


def test_order_ties_and_cross_series_hits():
    f = 3.0
    c = _cands([(5, 1, 9, 9.0, f), (3, 1, 9, 9.0, f + 0.1 / 50), (4, 2, 9, 9.0, f - 0.2 / 50), (9, 1, 1, 4.0, 40.0)])
    out = O.sift(c)
    assert out[0][0] == 1 and out[0][1:] == (3, 3, 5)      # series 3 ranks first among equal sigmas
    assert out[1][0] == 3 and out[1][1:] == (1, 9, 9)
