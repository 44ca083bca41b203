"""Pins of the FP64 oracle against things other than itself.

Each test checks one oracle step against a closed form, an identity, an
independent numerical method (mpmath quadrature of the defining integral,
exact rational arithmetic, a library routine) or brute force, so that a
dropped term, a flipped sign or index, or a transposed operand fails here.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle as O
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ----------------------------------------------------------------------------- spectrum

@pytest.mark.parametrize("N", [8, 10, 64, 250, 1024])
def test_dft_direct_matches_library_fft(N):
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N)
    a = O.dft_direct(x)
    b = O.spectrum(x)
    assert np.max(np.abs(a - b)) <= 1e-11 * np.sqrt(N) * np.max(np.abs(b))


def test_parseval():
    rng = np.random.default_rng(1)
    N = 1 << 12
    x = rng.standard_normal(N)
    A = O.spectrum(x)
    p = np.abs(A) ** 2
    lhs = np.sum(x * x)
    rhs = (p[0] + 2.0 * np.sum(p[1:N // 2]) + p[N // 2]) / N
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_pure_tone_at_integer_bin_is_exact():
    N, k0, a = 1 << 12, 137, 0.7
    n = np.arange(N)
    x = a * np.cos(2 * np.pi * k0 * n / N)
    A = O.spectrum(x)
    assert abs(abs(A[k0]) - N * a / 2) <= 1e-10 * N
    others = np.delete(np.abs(A), k0)
    assert others.max() <= 1e-10 * N


# ----------------------------------------------------------------------------- normalisation

def test_lower_median_on_hand_built_spectrum():
    # N = 16: bins k = 1..7 carry |A_k|^2 = 7, 1, 6, 2, 5, 3, 4 -> sorted 1..7,
    # lower median index floor((7-1)/2) = 3 -> value 4.
    A = np.zeros(9, dtype=complex)
    vals = [7, 1, 6, 2, 5, 3, 4]
    for k, v in enumerate(vals, start=1):
        A[k] = math.sqrt(v) * np.exp(1j * 0.3 * k)
    A[0] = 100.0
    A[8] = 50.0
    Ah, norm = O.normalise(A)
    assert norm == pytest.approx(4.0 / math.log(2.0), rel=1e-15)
    assert Ah[0] == 0 and Ah[8] == 0
    assert abs(Ah[3]) ** 2 == pytest.approx(6.0 * math.log(2.0) / 4.0, rel=1e-14)
    # even count: N = 10 -> bins 1..4, values 4,3,2,1 -> lower median index 1 -> value 2
    A = np.zeros(6, dtype=complex)
    A[1:5] = np.sqrt([4.0, 3.0, 2.0, 1.0])
    _, norm = O.normalise(A)
    assert norm == pytest.approx(2.0 / math.log(2.0), rel=1e-15)


def test_median_norm_of_white_noise_is_n_sigma2():
    rng = np.random.default_rng(7)
    N = 1 << 16
    for s in (1.0, 3.0):
        x = s * rng.standard_normal(N)
        _, norm = O.normalise(O.spectrum(x))
        assert norm / (N * s * s) == pytest.approx(1.0, abs=0.02)
    _, norm = O.normalise(O.spectrum(np.ones(N)), mode="fixed", fixed_var=2.5)
    assert norm == N * 2.5


# ----------------------------------------------------------------------------- response

RHO_POINTS = [(0.0, 0.5), (0.2, 0.5), (0.3, 7.5), (-3.7, 7.5), (10.5, -20.0), (0.0, 200.0),
              (99.5, 200.0), (150.0, 200.0), (0.5, 0.0), (-116.0, 2.0), (23.5, -150.0),
              (0.25, 0.002), (-7.0, 0.0005)]


def _rho_mp(q, z):
    """The defining integral by mpmath quadrature, split at every half turn of phase."""
    mpmath.mp.dps = 30
    q = mpmath.mpf(q)
    z = mpmath.mpf(z)
    f = lambda u: mpmath.expj(2 * mpmath.pi * (q * u + z * (u * u - u) / 2))
    npts = int(2 * (abs(float(q)) + abs(float(z)) / 2 + 2))
    pts = [mpmath.mpf(i) / npts for i in range(npts + 1)]
    v = mpmath.quad(f, pts)
    return complex(v)


@pytest.mark.parametrize("q,z", RHO_POINTS)
def test_rho_closed_form_matches_quadrature_of_definition(q, z):
    ref = _rho_mp(q, z)
    got = complex(O.rho(np.array([q]), z)[0])
    assert abs(got - ref) <= 2e-12, (q, z, got, ref)


def test_rho_quad_matches_closed_form():
    qs = np.linspace(-40, 40, 37)
    for z in (-30.0, -2.0, 0.7, 4.0, 60.0):
        a = O.rho(qs, z)
        b = O.rho_quad(qs, z)
        assert np.max(np.abs(a - b)) <= 1e-12


def test_rho_special_values_and_symmetries():
    assert complex(O.rho(np.array([0.5]), 0.0)[0]) == pytest.approx(2j / math.pi, abs=1e-15)
    assert abs(complex(O.rho(np.array([0.0]), 0.0)[0]) - 1.0) < 1e-15
    # integer offsets at z = 0 vanish: the DFT of an on-bin tone has one bin
    assert np.max(np.abs(O.rho(np.arange(1, 20), 0.0))) < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(20):
        q, z = rng.uniform(-50, 50), rng.uniform(0.1, 150)
        a = abs(O.rho(np.array([q]), z)[0])
        assert abs(O.rho(np.array([-q]), z)[0]) == pytest.approx(a, rel=1e-11)
        assert abs(O.rho(np.array([q]), -z)[0]) == pytest.approx(a, rel=1e-11)
    # continuity through z = 0 (closed form, quadrature and sinc branches)
    qs = np.linspace(-5, 5, 21)
    assert np.max(np.abs(O.rho(qs, 1e-7) - O.rho(qs, 0.0))) < 1e-6
    # the closed form (above 1e-3) and the quadrature (below) meet without a jump
    assert np.max(np.abs(O.rho(qs, 1e-3 * (1 + 1e-9)) - O.rho(qs, 1e-3 * (1 - 1e-9)))) < 1e-11


def test_rho_curvatures_at_peak():
    # |rho(q,0)|^2 = sinc^2 -> d2/dq2 = -2 pi^2 / 3; |rho(0,z)|^2 = 1 - pi^2 z^2 Var(u^2-u) + ...
    # with Var(u^2 - u) = 1/180 for u ~ U[0,1] -> d2/dz2 = -pi^2 / 90; no cross term.
    P = lambda q, z: abs(complex(O.rho(np.array([q]), z)[0])) ** 2
    h = 1e-3
    dqq = (P(h, 0) - 2 * P(0, 0) + P(-h, 0)) / h ** 2
    hz = 2e-2
    dzz = (P(0, hz) - 2 * P(0, 0) + P(0, -hz)) / hz ** 2
    dqz = (P(h, hz) - P(h, -hz) - P(-h, hz) + P(-h, -hz)) / (4 * h * hz)
    assert dqq == pytest.approx(-2 * math.pi ** 2 / 3, rel=1e-5)
    assert dzz == pytest.approx(-math.pi ** 2 / 90, rel=1e-4)
    assert abs(dqz) < 1e-6


def test_sampled_chirp_dft_matches_response():
    # DFT of the sampled signal of the single-series workload versus the
    # continuous-signal prediction (N a / 2) rho(r0 - k, z0): fixes the DFT
    # sign, the mean-frequency convention and the sign of z together.
    wl = synth.config1(noise=False)
    x = synth.generate(wl)[0].astype(np.float64)
    A = O.spectrum(x)
    inj = wl.injections[0]
    k = np.arange(9960, 10041)
    pred = 0.5 * wl.nsamp * inj.amp * O.rho(inj.r0 - k, inj.z0)
    peak = np.max(np.abs(pred))
    assert np.max(np.abs(A[k] - pred)) <= 1e-4 * peak
    flipped = 0.5 * wl.nsamp * inj.amp * O.rho(inj.r0 - k, -inj.z0)
    assert np.max(np.abs(A[k] - flipped)) > 0.1 * peak


# ----------------------------------------------------------------------------- plane

def _noise_spectrum(N, seed, mode="fixed"):
    rng = np.random.default_rng(seed)
    return O.normalise(O.spectrum(rng.standard_normal(N)), mode)[0]


def test_template_unit_energy_and_support():
    for z in (-20.0, -2.0, 0.0, 2.0, 7.0, 200.0):
        for p in (0, 1):
            d, t = O.template(z, p)
            m = O.half_width(z)
            assert d[0] == -m + p and d[-1] == m
            assert np.all(np.abs(p / 2 - d) <= m)
            assert np.sum(np.abs(t) ** 2) == pytest.approx(1.0, abs=1e-14)


def test_z0_row_at_integer_r_is_the_power_spectrum():
    N = 1 << 12
    Ah = _noise_spectrum(N, 11)
    rlo = 5
    pl = O.plane(Ah, rlo, 6.0, 2.0, method="direct")
    Z = 3
    k = np.arange(rlo, N // 2)
    assert np.max(np.abs(pl[Z, 2 * (k - rlo)] - np.abs(Ah[k]) ** 2)) <= 1e-12


def test_plane_fft_method_matches_direct_tap_sum():
    N = 1 << 12
    Ah = _noise_spectrum(N, 12)
    a = O.plane(Ah, 9, 20.0, 2.0, method="direct")
    b = O.plane(Ah, 9, 20.0, 2.0, method="fft")
    assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, a.max())


def test_plane_cells_match_full_plane():
    N = 1 << 11
    Ah = _noise_spectrum(N, 13)
    rlo, Z = 4, 5
    pl = O.plane(Ah, rlo, 10.0, 2.0)
    rng = np.random.default_rng(0)
    R = rng.integers(2 * rlo, N, 300)
    Zq = rng.integers(-Z, Z + 1, 300)
    v = O.plane_cells(Ah, R, Zq, 2.0)
    assert np.max(np.abs(v - pl[Zq + Z, R - 2 * rlo])) <= 1e-12


def test_white_noise_plane_cells_are_unit_exponential():
    N = 1 << 15
    Ah = _noise_spectrum(N, 21, "fixed")
    pl = O.plane(Ah, 30, 10.0, 2.0, method="fft")
    # cells 8 half-bins apart are nearly independent; compare with Exp(1)
    cells = pl[:, ::8].ravel()
    assert cells.mean() == pytest.approx(1.0, abs=0.02)
    assert stats.kstest(cells, "expon").pvalue > 1e-3


def _analytic_power(r, z, r0, z0, psig, K=16):
    """P_sig |sum_k rho(r0-k, z0) conj rho(r-k, z)|^2 / E over the trial's taps."""
    m = O.half_width(z, K)
    k = np.arange(math.ceil(r - m), math.floor(r + m) + 1)
    sig = np.array([_rho_mp(r0 - kk, z0) for kk in k])
    t = np.conj(O.rho(r - k, z))
    E = np.sum(np.abs(t) ** 2)
    return psig * abs(np.sum(sig * t)) ** 2 / E


def test_injected_sinusoid_recovered_at_analytic_power():
    wl = synth.config1(noise=False)
    inj = wl.injections[0]
    x = synth.generate(wl)[0]
    Ah, _ = O.normalise(O.spectrum(x), "fixed", 1.0)
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    psig = wl.nsamp * inj.amp ** 2 / 4.0
    assert psig == pytest.approx(81.92)
    for r, z in ((10000.5, 8.0), (10000.0, 6.0)):
        got = O.plane_cells(Ah, [int(2 * r)], [int(z / wl.dz)], wl.dz)[0]
        ref = _analytic_power(r, z, inj.r0, inj.z0, psig)
        assert got == pytest.approx(ref, rel=1e-4), (r, z, got, ref)


# ----------------------------------------------------------------------------- harmonics

def _round_half_up(fr: Fraction) -> int:
    return math.floor(fr + Fraction(1, 2))


def _round_half_away(fr: Fraction) -> int:
    s = 1 if fr >= 0 else -1
    return s * math.floor(abs(fr) + Fraction(1, 2))


def test_harmonic_index_matches_exact_rational_rounding():
    rng = np.random.default_rng(5)
    for H in (1, 2, 4, 8, 16, 32):
        R = rng.integers(0, 10 ** 7, 400)
        Zq = rng.integers(-150, 151, 400)
        for k in range(1, H + 1):
            Rk, Zk = O.harmonic_index(R, Zq, k, H)
            for i in range(0, 400, 37):
                assert Rk[i] == _round_half_up(Fraction(int(R[i]) * k, H))
                assert Zk[i] == _round_half_away(Fraction(int(Zq[i]) * k, H))
        Rk, Zk = O.harmonic_index(R, Zq, H, H)
        assert np.array_equal(Rk, R) and np.array_equal(Zk, Zq)


def test_stage_2h_even_harmonics_reproduce_stage_h():
    rng = np.random.default_rng(6)
    R = rng.integers(0, 10 ** 6, 1000)
    Zq = rng.integers(-100, 101, 1000)
    for H in (1, 2, 4, 8, 16):
        for k in range(1, H + 1):
            a = O.harmonic_index(R, Zq, k, H)
            b = O.harmonic_index(R, Zq, 2 * k, 2 * H)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_stage_maxima_match_brute_force_on_integer_plane():
    rng = np.random.default_rng(8)
    N, rlo, Z = 96, 2, 3
    pl = rng.integers(0, 50, size=(2 * Z + 1, N - 2 * rlo)).astype(np.float32)
    for H in (1, 2, 4, 8):
        R, M, Zs = O.stage_maxima(pl, rlo, Z, H, N)
        assert R[0] == 2 * rlo * H and R[-1] == N - 1
        for i, RR in enumerate(R):
            best, arg = None, None
            for zq in range(-Z, Z + 1):
                s = 0
                for k in range(1, H + 1):
                    rk = _round_half_up(Fraction(int(RR) * k, H))
                    zk = _round_half_away(Fraction(zq * k, H))
                    s += int(pl[zk + Z, rk - 2 * rlo])
                if best is None or s > best:
                    best, arg = s, zq
            assert M[i] == best and Zs[i] == arg


# ----------------------------------------------------------------------------- statistics

def test_threshold_closed_forms():
    for sigma in (3.0, 6.0, 8.5):
        p = 0.5 * math.erfc(sigma / math.sqrt(2))
        assert O.threshold(1, sigma) == pytest.approx(-math.log(p), rel=1e-13)
        T2 = O.threshold(2, sigma)
        assert math.exp(-T2) * (1 + T2) == pytest.approx(p, rel=1e-11)


def test_thresholds_match_high_precision_root():
    mpmath.mp.dps = 40
    sigma = 6
    p = mpmath.erfc(mpmath.mpf(sigma) / mpmath.sqrt(2)) / 2
    for H in (1, 2, 4, 8, 16, 32):
        T = mpmath.findroot(lambda t: mpmath.gammainc(H, t, mpmath.inf, regularized=True) - p,
                            H + 20)
        assert O.threshold(H, sigma) == pytest.approx(float(T), rel=1e-12)
        assert O.threshold(H, sigma) == pytest.approx(stats.gamma.isf(float(p), H), rel=1e-9)


def test_candidate_sigma_inverts_threshold():
    for H in (1, 2, 8, 32):
        for sigma in (2.0, 6.0, 12.0, 30.0):
            assert O.candidate_sigma(H, O.threshold(H, sigma)) == pytest.approx(sigma, rel=1e-9)
    # deep tail stays finite (log-space)
    assert O.candidate_sigma(1, 5000.0) == pytest.approx(math.sqrt(2 * 5000), rel=0.02)


# ----------------------------------------------------------------------------- end to end

def test_noise_free_single_series_candidates():
    """The injected sinusoid of the single-series workload, noise free, FIXED norm.

    The candidate set of the DFT path must equal the set of grid cells whose
    continuous-signal power exceeds T_1, and the grid maximum sits at
    (r, z) = (10000.5, 8) with the analytic power.
    """
    wl = synth.config1(noise=False)
    inj = wl.injections[0]
    x = synth.generate(wl)[0]
    cands = O.search_series(x, wl.tsamp, wl.zmax, wl.dz, 1, wl.sigma, norm="fixed", fixed_var=1.0)
    got = {(c["r_idx"], c["z_idx"]) for c in cands}
    assert got == {(20000, 4), (20001, 4), (20003, 1)}
    best = max(cands, key=lambda c: c["power"])
    assert (best["r_idx"], best["z_idx"]) == (20001, 4)
    psig = wl.nsamp * inj.amp ** 2 / 4
    assert best["power"] == pytest.approx(_analytic_power(10000.5, 8.0, inj.r0, inj.z0, psig),
                                          rel=1e-4)
    assert best["r_fund"] == 10000.5 and best["z_fund"] == 8.0
    assert best["f_hz"] == pytest.approx(10000.5 / (wl.nsamp * wl.tsamp))
    T1 = O.threshold(1, 6.0)
    # one candidate per r column: the column maximum over z decides, and its
    # smallest maximiser is reported
    Ah, _ = O.normalise(O.spectrum(x), "fixed", 1.0)
    R = np.arange(19990, 20012)
    cols = np.array([O.plane_cells(Ah, R, np.full(R.shape, zq), wl.dz) for zq in range(-10, 11)])
    rset = {r for r, _ in got}
    for i, RR in enumerate(R):
        assert (cols[:, i].max() > T1) == (int(RR) in rset)
        if int(RR) in rset:
            assert (int(RR), int(np.argmax(cols[:, i])) - 10) in got


def test_window_maxima_match_full_search():
    wl = synth.small_batch(1, 1 << 12, 1e-3, 10.0, 2.0, 4, config=91, signals=1,
                           amp_range=(0.3, 0.5))
    x = synth.generate(wl)[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    Ah, _ = O.normalise(O.spectrum(x))
    pl = O.plane(Ah, rlo, wl.zmax, wl.dz)
    Z = O.z_index_max(wl.zmax, wl.dz)
    for H in (1, 2, 4):
        R, M, Zs = O.stage_maxima(pl, rlo, Z, H, wl.nsamp)
        lo = 2 * rlo * H + 100
        Rw, Mw, Zw, _ = O.window_maxima(Ah, rlo, wl.zmax, wl.dz, H, lo, lo + 40)
        i0 = lo - 2 * rlo * H
        assert np.allclose(Mw, M[i0:i0 + 40], rtol=1e-12, atol=0)
        assert np.array_equal(Zw, Zs[i0:i0 + 40])


def test_plane_band_matches_full_plane_including_band_edges():
    # the banded direct sums equal the full plane column for column, also where the
    # taps run past bin 1 or bin N/2 - 1 and for a band that starts on an odd column
    N = 1 << 11
    Ah = _noise_spectrum(N, 14)
    rlo, zmax, dz = 3, 12.0, 2.0
    pl = O.plane(Ah, rlo, zmax, dz)
    for lo, hi in ((2 * rlo, 2 * rlo + 50), (2 * rlo + 7, 900), (N - 41, N)):
        pb = O.plane_band(Ah, lo, hi, zmax, dz)
        assert np.max(np.abs(pb - pl[:, lo - 2 * rlo:hi - 2 * rlo])) <= 1e-12
    Z = O.z_index_max(zmax, dz)
    rows = [0, 3, 2 * Z]
    pb = O.plane_band(Ah, 101, 333, zmax, dz, rows=rows)
    assert np.max(np.abs(pb[rows] - pl[rows, 101 - 2 * rlo:333 - 2 * rlo])) <= 1e-12
    assert not np.any(np.delete(pb, rows, axis=0))


def test_band_maxima_match_full_search():
    wl = synth.small_batch(1, 1 << 12, 1e-3, 10.0, 2.0, 8, config=92, signals=1,
                           amp_range=(0.3, 0.5))
    x = synth.generate(wl)[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    Ah, _ = O.normalise(O.spectrum(x))
    pl = O.plane(Ah, rlo, wl.zmax, wl.dz)
    Z = O.z_index_max(wl.zmax, wl.dz)
    for H in (1, 2, 4, 8):
        R, M, Zs = O.stage_maxima(pl, rlo, Z, H, wl.nsamp)
        for lo, hi in ((2 * rlo * H, 2 * rlo * H + 64), (2 * rlo * H + 333, wl.nsamp)):
            Rb, Mb, Zb = O.band_maxima(Ah, rlo, wl.zmax, wl.dz, H, lo, hi)
            i0 = lo - 2 * rlo * H
            assert np.array_equal(Rb, R[i0:i0 + hi - lo])
            assert np.allclose(Mb, M[i0:i0 + hi - lo], rtol=1e-12, atol=0)
            assert np.array_equal(Zb, Zs[i0:i0 + hi - lo])


def test_zero_series_normalises_to_zero_power():
    Ah, norm = O.normalise(O.spectrum(np.zeros(64)))
    assert norm == 0.0 and not np.any(Ah)
