"""Pins of the FP64 refinement oracle against mathematics it does not share code with.

* derivatives of rho: mpmath quadrature of the defining integrals, and central
  finite differences of the closed-form rho (scipy Fresnel);
* both evaluation branches (integration-by-parts identities, quadrature) agree;
* special case z = 0, integer r: the objective is the plain power |A^_k0|^2;
* objective gradients: central finite differences of the objective itself;
* a noise-free injected drifting sinusoid: the objective at the truth equals the
  continuum prediction N a^2/4 (sum over the window of |rho(r0 - k, z0)|^2)^2,
  and the ascent lands on the injected (r0, z0);
* the noisy single-series workload refines to within 0.1 bin and 1 drift bin;
* start points: brute force on a small plane.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import synth

PTS = [(0.3, 7.5), (-3.7, 7.5), (0.2, 0.5), (5.1, -3.0), (0.0, 0.0), (12.4, 1e-4), (30.2, 40.0),
       (2.5, 1.0), (-0.45, -0.999), (100.3, 150.0)]


def _mp_moments(q, z):
    f = lambda u, n: mp.exp(2j * mp.pi * (q * u + z * (u * u - u) / 2)) * u ** n
    nodes = mp.linspace(0, 1, int(abs(q) + abs(z) + 10))
    return [complex(mp.quad(lambda u: f(u, n), nodes)) for n in (0, 1, 2)]


@pytest.mark.parametrize("q,z", PTS)
def test_rho_derivatives_match_mpmath(q, z):
    mp.mp.dps = 30
    i0, i1, i2 = _mp_moments(q, z)
    r, dq, dz = O.rho_derivs(q, z)
    assert abs(r[0] - i0) <= 1e-13
    assert abs(dq[0] - 2j * math.pi * i1) <= 1e-12
    assert abs(dz[0] - 1j * math.pi * (i2 - i1)) <= 1e-12


@pytest.mark.parametrize("z", [2.0, -2.5, 3.0, 25.0])
def test_identity_and_quadrature_branches_agree(z):
    q = np.linspace(-30.3, 30.7, 23)
    r, dq, dz = O.rho_derivs(q, z)                      # |z| >= 1: identities
    i0, i1, i2 = O.rho_moments_quad(q, z)
    assert np.max(np.abs(r - i0)) <= 1e-12
    assert np.max(np.abs(dq - 2j * np.pi * i1)) <= 1e-11
    assert np.max(np.abs(dz - 1j * np.pi * (i2 - i1))) <= 1e-11


@pytest.mark.parametrize("q,z", [(0.3, 7.5), (4.2, 2.0), (-10.6, 31.0), (1.3, -5.0)])
def test_rho_derivatives_match_finite_differences_of_closed_form(q, z):
    h = 1e-5
    _, dq, dz = O.rho_derivs(q, z)
    fq = (O.rho(np.array([q + h]), z) - O.rho(np.array([q - h]), z)) / (2 * h)
    fz = (O.rho(np.array([q]), z + h) - O.rho(np.array([q]), z - h)) / (2 * h)
    assert abs(dq[0] - fq[0]) <= 1e-8
    assert abs(dz[0] - fz[0]) <= 1e-8


def _noise_spectrum(N, seed):
    rng = np.random.default_rng(seed)
    return O.normalise(O.spectrum(rng.standard_normal(N)))[0]


def test_zero_drift_integer_r_is_the_power_spectrum():
    Ah = _noise_spectrum(1 << 12, 1)
    for k0 in (5, 100, 2046):
        P, _, _, _ = O.refine_power(Ah, float(k0), 0.0, k0, 17)
        assert P == pytest.approx(abs(Ah[k0]) ** 2, rel=1e-12, abs=1e-14)


def test_objective_gradient_matches_finite_differences():
    Ah = _noise_spectrum(1 << 12, 2)
    rng = np.random.default_rng(3)
    h = 1e-3
    for _ in range(8):
        k0 = int(rng.integers(40, 1900))
        z = float(rng.uniform(-12, 12))
        r = k0 + float(rng.uniform(-0.9, 0.9))
        M = O.refine_window(z, 2.0)
        P, gr, gz, _ = O.refine_power(Ah, r, z, k0, M)
        fr = (O.refine_power(Ah, r + h, z, k0, M)[0] - O.refine_power(Ah, r - h, z, k0, M)[0]) / (2 * h)
        fz = (O.refine_power(Ah, r, z + h, k0, M)[0] - O.refine_power(Ah, r, z - h, k0, M)[0]) / (2 * h)
        assert abs(gr - fr) <= 1e-4 * (abs(fr) + P), (r, z, gr, fr)
        assert abs(gz - fz) <= 1e-4 * (abs(fz) + 0.1 * P), (r, z, gz, fz)


def test_spectrum_gradient_matches_finite_differences():
    Ah = _noise_spectrum(1 << 12, 4)
    k0, z, r = 700, 5.3, 700.37
    M = O.refine_window(z, 2.0)
    ks, g = O.refine_spec_grad(Ah, r, z, k0, M)
    P0 = O.refine_power(Ah, r, z, k0, M)[0]
    h = 1e-6
    for i in (0, M - 3, M, M + 1, 2 * M):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            A2 = Ah.copy()
            A2[ks[i]] += h * unit
            A3 = Ah.copy()
            A3[ks[i]] -= h * unit
            fd = (O.refine_power(A2, r, z, k0, M)[0] - O.refine_power(A3, r, z, k0, M)[0]) / (2 * h)
            assert abs(part(g[i]) - fd) <= 1e-6 * (abs(fd) + P0)


def test_noise_free_injection_refines_to_the_truth():
    wl = synth.config1(noise=False)
    inj = wl.injections[0]
    Ah = O.normalise(O.spectrum(synth.generate(wl)[0]), "fixed", 1.0)[0]
    k0 = int(round(inj.r0))
    M = O.refine_window(inj.z0, wl.dz)
    ks = np.arange(k0 - M, k0 + M + 1)
    energy = float(np.sum(np.abs(O.rho(inj.r0 - ks, inj.z0)) ** 2))
    predicted = wl.nsamp * inj.amp ** 2 / 4.0 * energy ** 2          # continuum model of the DFT
    P_true = O.refine_power(Ah, inj.r0, inj.z0, k0, M)[0]
    assert P_true == pytest.approx(predicted, rel=2e-3)
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    pl = O.plane(Ah, rlo, wl.zmax, wl.dz, method="fft")
    R, Zq = O.refine_starts(pl, rlo, O.z_index_max(wl.zmax, wl.dz), 4)[0]
    assert (R, Zq) == (20000, 4)
    r, z, P = O.refine(Ah, R / 2, Zq * wl.dz, wl.dz)
    assert abs(r - inj.r0) <= 0.01 and abs(z - inj.z0) <= 0.05, (r, z)
    assert P >= P_true * (1 - 1e-6)
    _, gr, gz, _ = O.refine_power(Ah, r, z, int(round(R / 2)), O.refine_window(Zq * wl.dz, wl.dz))
    assert abs(gr) <= 1e-3 * P and abs(gz) <= 1e-3 * P         # a stationary point


def test_noisy_single_series_refines_near_the_injection():
    wl = synth.config1()
    inj = wl.injections[0]
    Ah = O.normalise(O.spectrum(synth.generate(wl)[0]))[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    pl = O.plane(Ah, rlo, wl.zmax, wl.dz, method="fft")
    starts = O.refine_starts(pl, rlo, O.z_index_max(wl.zmax, wl.dz), 4096)
    assert len(starts) == 4096
    near = [s for s in starts if abs(s[0] / 2 - inj.r0) <= 1 and abs(s[1] * wl.dz - inj.z0) <= 2 * wl.dz]
    assert near, "no start next to the injected signal"
    r, z, P = O.refine(Ah, near[0][0] / 2, near[0][1] * wl.dz, wl.dz)
    assert abs(r - inj.r0) <= 0.1 and abs(z - inj.z0) <= 1.0, (r, z, P)


def test_ascent_stays_inside_its_clamp():
    Ah = _noise_spectrum(1 << 13, 5)
    rng = np.random.default_rng(6)
    for _ in range(6):
        r0 = float(rng.integers(50, 4000))
        z0 = float(2 * rng.integers(-5, 6))
        r, z, P = O.refine(Ah, r0, z0, 2.0)
        assert abs(r - r0) <= 1.0 + 1e-12 and abs(z - z0) <= 4.0 + 1e-12
        k0 = int(r0)
        assert P >= O.refine_power(Ah, r0, z0, k0, O.refine_window(z0, 2.0))[0] * 0.999


def test_start_points_by_brute_force():
    rng = np.random.default_rng(7)
    NZ, NR, rlo, Z = 7, 40, 3, 3
    pl = rng.integers(0, 6, (NZ, NR)).astype(float)          # many ties
    got = O.refine_starts(pl, rlo, Z, 1000)
    sub = pl[:, 0::2]
    cands = []
    for zi in range(NZ):
        for j in range(sub.shape[1]):
            ok = True
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy or dx) and 0 <= zi + dy < NZ and 0 <= j + dx < sub.shape[1]:
                        v = sub[zi + dy, j + dx]
                        earlier = dx < 0 or (dx == 0 and dy < 0)
                        if (earlier and not sub[zi, j] > v) or (not earlier and not sub[zi, j] >= v):
                            ok = False
            if ok:
                cands.append((-sub[zi, j], j, zi))
    cands.sort()
    assert got == [(2 * rlo + 2 * j, zi - Z) for _, j, zi in cands]
