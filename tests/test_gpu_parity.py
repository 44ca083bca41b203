"""HIP path versus the FP64 oracle at sizes the oracle finishes in seconds.

Every case spans several overlap-save segments and harmonic-sum tiles and
ends in a ragged tail (the last segment and tile are partial).
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from fdas_check import OracleSeries, assert_candidates_match, assert_plane_close

pytestmark = pytest.mark.gpu


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _noise(B, N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, N)).astype(np.float32)


# ----------------------------------------------------------------------------- spectrum

SPECTRUM_LENGTHS = [
    8, 64, 1 << 12, 1 << 14, 1 << 15, 1 << 17, 1 << 23,       # one workgroup up to 2^14, four-step above
    12, 30, 4374, 12000,                                      # N/2 = 6, 15, 3^7, 2^4 3 5^3: in one workgroup
    31250, 153600, 6291456,                                   # N/2 = 5^6, 2^10 3 5^2, 3 2^20: four-step
    33592320,                                                 # N/2 = 2^9 3^8 5: rows of 4320, split pass
]


@pytest.mark.parametrize("N", SPECTRUM_LENGTHS)
def test_spectrum_and_median_norm(fdas_gpu, N):
    B = 3 if N < (1 << 22) else 2
    x = _noise(B, N, N)
    x[1] *= 5.0
    plan = fdas_gpu.Plan(N, B, 0.0, 2.0, 1, flo_hz=0.0)
    A, norm = plan.spectrum(_cuda(x))
    A = A.cpu().numpy().astype(np.complex128)
    for b in range(B):
        ref = O.spectrum(x[b])
        err = np.max(np.abs(A[b] - ref)) / np.max(np.abs(ref))
        assert err < 3e-6, (b, err)
        _, nref = O.normalise(ref)
        assert norm[b] == pytest.approx(nref, rel=2e-5)


# ----------------------------------------------------------------------------- plane

PLANE_CASES = [
    # (N, tsamp, zmax, dz, K, seg_len)
    (1 << 12, 1e-3, 0.0, 2.0, 16, 0),        # one z row, L = 512
    (1 << 13, 1e-3, 10.0, 2.0, 16, 0),       # L = 512, many segments
    (1 << 13, 1e-3, 10.0, 2.0, 8, 1024),     # forced L = 1024, other K
    (1 << 14, 1e-3, 40.0, 1.0, 16, 0),       # 81 rows, L = 1024, four z groups
    (1 << 14, 1e-3, 200.0, 2.0, 16, 0),      # 201 rows, L = 2048, eight z groups
    (1 << 14, 1e-3, 300.0, 4.0, 16, 0),      # L = 4096
]


@pytest.mark.parametrize("case", PLANE_CASES, ids=lambda c: f"N{c[0]}-z{c[2]}-dz{c[3]}-K{c[4]}-L{c[5]}")
def test_plane_matches_oracle(fdas_gpu, case):
    N, ts, zmax, dz, K, L = case
    B = 2
    wl = synth.small_batch(B, N, ts, zmax, dz, 1, config=92, signals=2, amp_range=(0.2, 0.6))
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(N, B, zmax, dz, 1, K=K, seg_len=L)
    P = plan.plane(_cuda(x), ts).cpu().numpy()
    rlo = O.rlo_bins(N, ts)
    for b in range(B):
        Ah, _ = O.normalise(O.spectrum(x[b]))
        ref = O.plane(Ah, rlo, zmax, dz, K, method="fft")
        assert_plane_close(P[b], ref)


def test_plane_single_series_workload(fdas_gpu):
    wl = synth.config1()
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1)
    P = plan.plane(_cuda(x), wl.tsamp).cpu().numpy()[0]
    Ah, _ = O.normalise(O.spectrum(x[0]))
    ref = O.plane(Ah, O.rlo_bins(wl.nsamp, wl.tsamp), wl.zmax, wl.dz, method="direct")
    assert_plane_close(P, ref)


def test_plane_fixed_norm_noise_free_peak(fdas_gpu):
    wl = synth.config1(noise=False)
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1, norm="fixed", fixed_var=1.0)
    P = plan.plane(_cuda(x), wl.tsamp).cpu().numpy()[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    # grid maximum of the injected sinusoid at (r, z) = (10000.5, 8)
    zi, c = np.unravel_index(np.argmax(P), P.shape)
    assert (zi - 10, c + 2 * rlo) == (4, 20001)
    assert P[zi, c] == pytest.approx(70.258485, rel=1e-4)


# ----------------------------------------------------------------------------- harmonic sums

@pytest.mark.parametrize("bound", [0, 1], ids=["bounded", "exhaustive"])
@pytest.mark.parametrize("numharm", [1, 2, 4, 8, 16, 32])
def test_harmsum_bit_exact_on_integer_planes(fdas_gpu, numharm, bound):
    import torch
    B, N, ts, zmax, dz = 3, 1 << 12, 1e-2, 6.0, 2.0
    rlo = O.rlo_bins(N, ts)
    Z = O.z_index_max(zmax, dz)
    rng = np.random.default_rng(100 + numharm)
    planes = rng.integers(0, 40, size=(B, 2 * Z + 1, N - 2 * rlo)).astype(np.float32)
    # a few strong integer peaks so that high stages pass their thresholds too
    for b in range(B):
        for _ in range(20):
            planes[b, rng.integers(0, 2 * Z + 1), rng.integers(0, N - 2 * rlo)] = rng.integers(100, 4000)
    sigma = 6.0
    plan = fdas_gpu.Plan(N, B, zmax, dz, numharm, harm_bound=bound)
    g = plan.harmsum(torch.from_numpy(planes).cuda(), N, ts, sigma=sigma, cap=1 << 18)
    got = sorted((int(c["series"]), int(c["harm"]), int(c["r_idx"]), int(c["z_idx"]), float(c["power"]))
                 for c in g)
    ref = []
    for b in range(B):
        orc = OracleSeries(np.zeros(N), ts, zmax, dz, numharm, plane=planes[b])
        for H, R, Zq, M in orc.candidates(sigma):
            ref.append((b, H, R, Zq, M))
    ref.sort()
    assert len(ref) > 100
    assert got == ref


# ----------------------------------------------------------------------------- search

def test_search_single_series_workload(fdas_gpu):
    wl = synth.config1()
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, wl.numharm)
    g = plan.search(_cuda(x), wl.tsamp, sigma=wl.sigma)
    orc = OracleSeries(x[0], wl.tsamp, wl.zmax, wl.dz, wl.numharm, method="direct")
    common, _ = assert_candidates_match(g, {0: orc}, wl.sigma)
    assert common >= 1
    best = g[np.argmax(g["power"])]
    assert abs(best["r_fund"] - 10000.3) <= 1.0 and abs(best["z_fund"] - 7.5) <= 2.0


def test_search_noise_free_fixed_norm_three_candidates(fdas_gpu):
    wl = synth.config1(noise=False)
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1, norm="fixed", fixed_var=1.0)
    g = plan.search(_cuda(x), wl.tsamp, sigma=6.0)
    assert [(int(c["r_idx"]), int(c["z_idx"])) for c in g] == [(20000, 4), (20001, 4), (20003, 1)]
    assert g["power"][1] == pytest.approx(70.258485, rel=1e-4)
    assert g["sigma"][1] == pytest.approx(O.candidate_sigma(1, g["power"][1]), rel=1e-5)
    assert g["f_hz"][1] == pytest.approx(10000.5 / (wl.nsamp * wl.tsamp), rel=1e-12)
    assert g["fdot_hz_s"][1] == pytest.approx(8.0 / (wl.nsamp * wl.tsamp) ** 2, rel=1e-12)


SEARCH_CASES = [
    # (B, N, tsamp, zmax, dz, numharm, sigma)
    (4, 1 << 14, 1e-3, 20.0, 2.0, 4, 6.0),
    (3, 1 << 15, 5e-4, 50.0, 2.0, 8, 6.0),
    (2, 1 << 14, 1e-3, 200.0, 2.0, 16, 5.0),
    (2, 1 << 13, 2e-3, 10.0, 1.0, 32, 4.0),
    (2, 1 << 13, 1e-3, 0.0, 2.0, 8, 3.0),
]


@pytest.mark.parametrize("case", SEARCH_CASES, ids=lambda c: f"B{c[0]}-N{c[1]}-z{c[3]}-h{c[5]}-s{c[6]}")
def test_search_matches_oracle(fdas_gpu, case):
    B, N, ts, zmax, dz, nh, sigma = case
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, sigma=sigma, config=93, signals=B,
                           amp_range=(0.3, 1.0))
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(N, B, zmax, dz, nh)
    g = plan.search(_cuda(x), ts, sigma=sigma, cap=1 << 18)
    oracles = {b: OracleSeries(x[b], ts, zmax, dz, nh, method="fft") for b in range(B)}
    common, banded = assert_candidates_match(g, oracles, sigma)
    assert common >= 1


SMOOTH_CASES = [
    # (B, N, tsamp, zmax, dz, numharm, sigma): N/2 = 2^4 3 5^3 (one workgroup FFT) and
    # 2^10 3 5^2 (four-step FFT)
    (2, 12000, 1e-3, 20.0, 2.0, 4, 5.0),
    (2, 153600, 2e-4, 50.0, 2.0, 8, 6.0),
]


@pytest.mark.parametrize("case", SMOOTH_CASES, ids=lambda c: f"B{c[0]}-N{c[1]}-z{c[3]}-h{c[5]}")
def test_search_5smooth_lengths_match_oracle(fdas_gpu, case):
    B, N, ts, zmax, dz, nh, sigma = case
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, sigma=sigma, config=83, signals=B, amp_range=(0.3, 1.0))
    x = synth.generate(wl)
    plan = fdas_gpu.Plan(N, B, zmax, dz, nh)
    g = plan.search(_cuda(x), ts, sigma=sigma, cap=1 << 18)
    oracles = {b: OracleSeries(x[b], ts, zmax, dz, nh, method="fft") for b in range(B)}
    common, _ = assert_candidates_match(g, oracles, sigma)
    assert common >= 1
    P = plan.plane(_cuda(x), ts).cpu().numpy()
    for b in range(B):
        assert_plane_close(P[b], oracles[b].plane)


def test_search_chunked_workspace_matches_unchunked(fdas_gpu):
    B, N, ts, zmax, dz, nh = 5, 1 << 13, 1e-3, 20.0, 2.0, 4
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, config=94, signals=3)
    x = _cuda(synth.generate(wl))
    full = fdas_gpu.Plan(N, B, zmax, dz, nh).search(x, ts, sigma=4.0, cap=1 << 18)
    rows = 2 * O.z_index_max(zmax, dz) + 1
    small = fdas_gpu.Plan(N, B, zmax, dz, nh, max_workspace_bytes=2 * rows * N * 4,
                          max_candidates=64).search(x, ts, sigma=4.0, cap=1 << 18)
    assert len(full) > 64
    assert np.array_equal(full, small)


# ----------------------------------------------------------------------------- edge cases

# bound of the FP32 device significance against the FP64 host statistics
SIGMA_TOL = 1e-5


def test_device_significance_equals_host_statistics(fdas_gpu):
    """Record sigmas are computed on the device in FP32; they agree with the FP64
    host statistics (and so with the oracle's reading) within 1e-5 (relative, or
    absolute below 1) for every stage, from powers just above a low threshold to
    the 10^5-10^6 of strong tones."""
    B, N, ts, zmax, dz, nh = 3, 1 << 14, 1e-3, 20.0, 2.0, 32
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, config=99, signals=2, amp_range=(0.3, 3.0))
    x = synth.generate(wl)
    # a strong on-bin tone in the last series: powers near N a^2 / 4 = 1.5e5
    x[2] += (6.0 * np.cos(2 * np.pi * 1234.0 * np.arange(N) / N)).astype(np.float32)
    c = fdas_gpu.Plan(N, B, zmax, dz, nh).search(_cuda(x), ts, sigma=2.5, cap=1 << 20)
    assert len(c) > 1000 and len(set(c["harm"].tolist())) == 6
    assert c["power"].max() > 1e5
    host = np.array([fdas_gpu.sigma_of(int(h), float(p)) for h, p in zip(c["harm"], c["power"])])
    np.testing.assert_allclose(c["sigma"], host, rtol=SIGMA_TOL, atol=SIGMA_TOL)
    for i in np.linspace(0, len(c) - 1, 25).astype(int):
        ref = O.candidate_sigma(int(c["harm"][i]), float(c["power"][i]))
        assert c["sigma"][i] == pytest.approx(ref, rel=SIGMA_TOL, abs=SIGMA_TOL)


def test_zero_series_give_no_candidates(fdas_gpu):
    N = 1 << 12
    x = np.zeros((2, N), dtype=np.float32)
    x[1] = _noise(1, N, 5)[0]
    plan = fdas_gpu.Plan(N, 2, 10.0, 2.0, 4)
    g = plan.search(_cuda(x), 1e-3, sigma=3.0)
    assert not np.any(g["series"] == 0)


def test_truncation_reports_true_count(fdas_gpu):
    N = 1 << 13
    x = _noise(2, N, 7)
    plan = fdas_gpu.Plan(N, 2, 10.0, 2.0, 2)
    full = plan.search(_cuda(x), 1e-3, sigma=2.0, cap=1 << 16)
    assert len(full) > 50
    part, total = plan.search(_cuda(x), 1e-3, sigma=2.0, cap=17, allow_trunc=True)
    assert total == len(full)
    assert np.array_equal(part, full[:17])
    whole, total = plan.search(_cuda(x), 1e-3, sigma=2.0, cap=1 << 16, allow_trunc=True)
    assert total == len(full) and np.array_equal(whole, full)


def test_results_of_earlier_calls_are_not_overwritten(fdas_gpu):
    # every call returns records in storage of its own: a later search on the
    # same plan (other data, other threshold, more records) leaves them intact
    N = 1 << 13
    plan = fdas_gpu.Plan(N, 2, 10.0, 2.0, 4)
    x1, x2 = _cuda(_noise(2, N, 21)), _cuda(_noise(2, N, 22))
    first = plan.search(x1, 1e-3, sigma=3.0)
    kept = first.copy()
    second = plan.search(x2, 1e-3, sigma=2.0)
    part, _ = plan.search(x2, 1e-3, sigma=2.0, cap=5, allow_trunc=True)
    assert len(second) > len(first) > 0
    assert np.array_equal(first, kept)
    assert np.array_equal(part, second[:5])
    again = plan.search(x1, 1e-3, sigma=3.0)
    assert np.array_equal(again, kept)


def test_invalid_arguments_return_status(fdas_gpu):
    F = fdas_gpu
    N = 1 << 12
    x = _cuda(_noise(2, N, 9))
    plan = F.Plan(N, 2, 10.0, 2.0, 4)
    bad = [dict(zmax=11.0), dict(numharm=8), dict(numharm=3), dict(sigma=0.0), dict(sigma=float("nan")),
           dict(tsamp=0.0), dict(tsamp=10.0)]
    for kw in bad:
        args = dict(tsamp=1e-3, zmax=10.0, dz=2.0, numharm=4, sigma=6.0)
        args.update(kw)
        with pytest.raises(F.FdasError) as e:
            plan.search(x, **args)
        assert e.value.status == F.FDAS_E_INVAL, kw
    big = _cuda(_noise(1, 2 * N, 1))
    with pytest.raises(F.FdasError) as e:
        plan.search(big, 1e-3)
    assert e.value.status == F.FDAS_E_INVAL
    with pytest.raises(F.FdasError) as e:
        plan.search(_cuda(_noise(3, N, 1)), 1e-3)
    assert e.value.status == F.FDAS_E_INVAL
    odd = F.Plan(N, 2, 10.0, 2.0, 4)
    with pytest.raises(F.FdasError) as e:
        odd.search(_cuda(_noise(1, N - 24, 1)), 1e-3)
    assert e.value.status == F.FDAS_E_UNSUPPORTED
    # the plan still works after rejected calls
    assert plan.search(x, 1e-3, sigma=6.0) is not None


def test_harmonic_sum_tile_orders_give_identical_results(fdas_gpu):
    B, N, ts, zmax, dz, nh = 3, 1 << 14, 1e-3, 40.0, 2.0, 8
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, config=95, signals=3, amp_range=(0.3, 1.0))
    x = _cuda(synth.generate(wl))
    res = [fdas_gpu.Plan(N, B, zmax, dz, nh, harm_order=o).search(x, ts, sigma=3.0, cap=1 << 18)
           for o in (0, 1, 2, 3)]
    assert len(res[0]) > 20
    for r in res[1:]:
        assert np.array_equal(res[0], r)


BOUND_CASES = [
    # (B, N, tsamp, zmax, dz, numharm, sigma, block)
    (3, 1 << 14, 1e-3, 40.0, 2.0, 8, 6.0, 0),
    (3, 1 << 14, 1e-3, 40.0, 2.0, 8, 3.0, 0),     # low threshold: most blocks summed exactly
    (2, 1 << 14, 1e-3, 200.0, 2.0, 16, 5.0, 0),
    (2, 1 << 13, 2e-3, 10.0, 1.0, 32, 4.0, 0),
    (2, 1 << 13, 1e-3, 0.0, 2.0, 4, 4.0, 0),      # one drift row
    (2, 1 << 14, 1e-3, 60.0, 2.0, 8, 5.0, 1),     # one row per block
    (2, 1 << 14, 1e-3, 60.0, 2.0, 8, 5.0, 61),    # one block per z group
    (2, 1 << 14, 1e-3, 100.0, 2.0, 8, 4.0, 6),    # a fraction range over three row blocks
]


@pytest.mark.parametrize("case", BOUND_CASES, ids=lambda c: f"N{c[1]}-z{c[3]}-h{c[5]}-s{c[6]}-bz{c[7]}")
def test_bounded_harmonic_sums_equal_exhaustive(fdas_gpu, case):
    B, N, ts, zmax, dz, nh, sigma, bz = case
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, sigma=sigma, config=96, signals=B,
                           amp_range=(0.3, 1.0))
    x = _cuda(synth.generate(wl))
    ref = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_bound=1).search(x, ts, sigma=sigma, cap=1 << 18)
    got = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_block=bz).search(x, ts, sigma=sigma, cap=1 << 18)
    assert len(ref) > 5
    if not np.array_equal(ref, got):
        kr = {tuple(int(v) for v in (c["series"], c["harm"], c["r_idx"], c["z_idx"])): float(c["power"]) for c in ref}
        kg = {tuple(int(v) for v in (c["series"], c["harm"], c["r_idx"], c["z_idx"])): float(c["power"]) for c in got}
        only_r = sorted(set(kr) - set(kg))[:10]
        only_g = sorted(set(kg) - set(kr))[:10]
        diff = [(k, kr[k], kg[k]) for k in sorted(set(kr) & set(kg)) if kr[k] != kg[k]][:10]
        raise AssertionError(f"exhaustive only {only_r}; bounded only {only_g}; power differs {diff}")


@pytest.mark.parametrize("numharm,bz", [(8, 0), (16, 0), (32, 0), (32, 3), (4, 1)])
def test_bounded_harmsum_bit_exact_on_the_same_float_plane(fdas_gpu, numharm, bz):
    """Bounded and exhaustive harmonic sums of one caller plane give identical records."""
    import torch
    B, N, ts, zmax, dz = 2, 1 << 14, 1e-3, 30.0, 2.0
    wl = synth.small_batch(B, N, ts, zmax, dz, numharm, config=97, signals=B, amp_range=(0.3, 1.0))
    x = _cuda(synth.generate(wl))
    P = fdas_gpu.Plan(N, B, zmax, dz, numharm).plane(x, ts)
    sig = 3.5
    ref = fdas_gpu.Plan(N, B, zmax, dz, numharm, harm_bound=1).harmsum(P, N, ts, sigma=sig, cap=1 << 18)
    got = fdas_gpu.Plan(N, B, zmax, dz, numharm, harm_block=bz).harmsum(P, N, ts, sigma=sig, cap=1 << 18)
    assert len(ref) > 20
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("harm_pair", [0, 1], ids=["maxima-per-bin", "maxima-per-column"])
def test_bounded_harmsum_exact_near_thresholds_and_at_half_precision_extremes(fdas_gpu, harm_pair):
    """Block maxima are stored as halves rounded up: cells a fraction of a half ulp
    above (or around) a stage threshold, powers beyond the largest half and
    powers below the smallest normal half must not change any candidate."""
    import torch
    B, N, ts, zmax, dz, nh, sigma = 2, 1 << 14, 1e-3, 30.0, 2.0, 8, 6.0
    rlo = O.rlo_bins(N, ts)
    Z = O.z_index_max(zmax, dz)
    NZ, NR = 2 * Z + 1, N - 2 * rlo
    rng = np.random.default_rng(4242)
    P = (rng.exponential(1.0, (B, NZ, NR)) * 10.0 ** rng.uniform(-9.0, 0.0, (B, NZ, NR))).astype(np.float32)
    T = {H: np.float32(O.threshold(H, sigma)) for H in (1, 2, 4, 8)}
    for b in range(B):
        # stage 1: single cells at the next float above T_1, or within 2^-10 of it
        rows = rng.integers(0, NZ, 400)
        cols = rng.integers(0, NR, 400)
        vals = (T[1] * (1.0 + rng.uniform(-2.0 ** -10, 2.0 ** -10, 400))).astype(np.float32)
        vals[:100] = np.nextafter(T[1], np.float32(np.inf))
        P[b, rows, cols] = vals
        # stage 8 on the zero-drift row: all eight harmonics near T_8 / 8
        for R in rng.integers(2 * rlo * 8, N, 150):
            u = np.float32(T[8] / 8.0 * (1.0 + rng.uniform(-2.0 ** -10, 2.0 ** -10)))
            for k in range(1, 9):
                P[b, Z, (2 * int(R) * k + 8) // 16 - 2 * rlo] = u
        # beyond the largest finite half
        P[b, rng.integers(0, NZ, 5), rng.integers(0, NR, 5)] = np.float32([7e4, 1e6, 1e9, 1e20, 1e30])
    Pt = torch.from_numpy(P).cuda()
    ref = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_bound=1).harmsum(Pt, N, ts, sigma=sigma, cap=1 << 18)
    got = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_pair=harm_pair).harmsum(Pt, N, ts, sigma=sigma, cap=1 << 18)
    assert len(ref) > 400
    assert np.array_equal(ref, got)


def test_bounded_search_exact_with_powers_beyond_the_largest_half(fdas_gpu):
    """Strong signals make plane powers far above 65504 (maxima stored as +inf)."""
    B, N, ts, zmax, dz, nh = 2, 1 << 14, 1e-3, 40.0, 2.0, 8
    rng = np.random.default_rng(98)
    t = np.arange(N) * ts
    T = N * ts
    x = rng.standard_normal((B, N))
    for b, (f, z, amp) in enumerate([(101.3, 12.0, 40.0), (37.77, -30.0, 25.0)]):
        # drifting sinusoid: z bins of frequency drift over the observation
        x[b] += amp * np.cos(2 * np.pi * (f * t + 0.5 * z / T ** 2 * t ** 2))
    x = _cuda(x.astype(np.float32))
    plan = fdas_gpu.Plan(N, B, zmax, dz, nh)
    P = plan.plane(x, ts)
    assert float(P.max()) > 1e5
    ref = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_bound=1).search(x, ts, sigma=6.0, cap=1 << 18)
    got = plan.search(x, ts, sigma=6.0, cap=1 << 18)
    assert len(ref) > 5
    assert np.array_equal(ref, got)


def test_bounded_search_exact_when_thresholds_pass_the_code_range(fdas_gpu):
    """Per-column block maxima are 8-bit codes that saturate at 252: with a
    stage threshold at or above that (high sigma) a saturated bound could not
    be told from a candidate, so every block is summed exactly; the records
    still equal those of the exhaustive sums."""
    B, N, ts, zmax, dz, nh, sigma = 2, 1 << 14, 1e-3, 40.0, 2.0, 16, 20.0
    assert fdas_gpu.threshold(16, sigma) >= 252.0 > fdas_gpu.threshold(8, sigma)
    rng = np.random.default_rng(99)
    t = np.arange(N) * ts
    T = N * ts
    x = rng.standard_normal((B, N))
    for b, (f, z, amp) in enumerate([(61.9, 8.0, 60.0), (143.21, -24.0, 45.0)]):
        x[b] += amp * np.cos(2 * np.pi * (f * t + 0.5 * z / T ** 2 * t ** 2))
    x = _cuda(x.astype(np.float32))
    ref = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_bound=1).search(x, ts, sigma=sigma, cap=1 << 18)
    got = fdas_gpu.Plan(N, B, zmax, dz, nh, harm_pair=1).search(x, ts, sigma=sigma, cap=1 << 18)
    assert len(ref) > 5
    assert np.array_equal(ref, got)
