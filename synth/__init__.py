"""Seeded synthetic inputs for the acceleration search.

This module generates dedispersed-time-series-shaped float32 inputs and
their ground truth. It holds none of the search's arithmetic (no Fourier
transform, no response template, no harmonic sum, no threshold): both the
FP64 oracle tests and the HIP path tests draw their inputs from here, so
that each side sees the same bytes.

Workload shapes follow the paper's test files (Table 1: a 52.4288 s FAST
drift-scan file sampled at 0.2 ms, a 2100.224 s PMPS file) and its
dedispersion plans (Tables 2-3), with white Gaussian noise standing in for
the missing survey data.

Signal model (stated here because generator and searches must agree on it):
a sinusoid whose Fourier frequency, in bins of 1/T, is r0 at mid-observation
and drifts by z0 bins over the observation, i.e. the phase in cycles is
    phi(u) = phi0 + r0*u + z0*(u*u - u)/2,   u = n/N in [0, 1).
Pulse trains replace cos(2 pi phi) by a von Mises profile of the same phase.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 191212807


def seed_for(config: int, series: int) -> int:
    """Seed of one series: one PCG64 stream per (config, series)."""
    return BASE_SEED + 1000 * int(config) + int(series)


@dataclasses.dataclass
class Injection:
    series: int
    kind: str            # "sine" | "pulse" | "tone"
    r0: float            # fundamental Fourier frequency at mid-observation (bins)
    z0: float            # fundamental drift over the observation (bins)
    amp: float           # sine amplitude or pulse peak amplitude
    duty: float = 0.0    # pulse FWHM as a fraction of the period
    phase0: float = 0.0  # cycles

    def as_dict(self):
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    nsamp: int
    nseries: int
    tsamp: float
    zmax: float
    dz: float
    numharm: int
    sigma: float
    injections: List[Injection]
    noise: bool = True
    series_idx: Optional[List[int]] = None   # which series of the batch were generated

    @property
    def tobs(self) -> float:
        return self.nsamp * self.tsamp


def _chirp_phase(n: int, r0: float, z0: float, phase0: float) -> np.ndarray:
    u = np.arange(n, dtype=np.float64) / n
    return phase0 + r0 * u + z0 * (u * u - u) * 0.5


def add_sine(x: np.ndarray, r0: float, z0: float, amp: float, phase0: float = 0.0) -> None:
    """x += amp*cos(2 pi phi(u)), summed in FP64."""
    ph = _chirp_phase(x.shape[-1], r0, z0, phase0)
    x += amp * np.cos(2.0 * np.pi * ph)


def von_mises_kappa(duty: float) -> float:
    """Concentration whose profile exp(kappa(cos 2 pi phi - 1)) has FWHM = duty."""
    return math.log(2.0) / (1.0 - math.cos(math.pi * duty))


def add_pulse(x: np.ndarray, r0: float, z0: float, amp: float, duty: float, phase0: float = 0.0) -> None:
    """x += amp*exp(kappa(cos 2 pi phi(u) - 1)), a pulse train of the given FWHM duty."""
    ph = _chirp_phase(x.shape[-1], r0, z0, phase0)
    kappa = von_mises_kappa(duty)
    x += amp * np.exp(kappa * (np.cos(2.0 * np.pi * ph) - 1.0))


def _series(nsamp: int, seed: int, noise: bool) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    if noise:
        return rng.standard_normal(nsamp)
    return np.zeros(nsamp, dtype=np.float64)


def _render(wl: Workload, series_idx) -> np.ndarray:
    out = np.empty((len(series_idx), wl.nsamp), dtype=np.float32)
    by_series = {}
    for inj in wl.injections:
        by_series.setdefault(inj.series, []).append(inj)
    for row, b in enumerate(series_idx):
        x = _series(wl.nsamp, seed_for(wl.config, b), wl.noise)
        for inj in by_series.get(b, []) + by_series.get(-1, []):
            if inj.kind in ("sine", "tone"):
                add_sine(x, inj.r0, inj.z0, inj.amp, inj.phase0)
            elif inj.kind == "pulse":
                add_pulse(x, inj.r0, inj.z0, inj.amp, inj.duty, inj.phase0)
            else:
                raise ValueError(inj.kind)
        out[row] = x.astype(np.float32)
    return out


# --------------------------------------------------------------------------- configs

def config1(noise: bool = True) -> Workload:
    """One FAST-like series: 2^17 samples at 0.2 ms, a sinusoid at r0=10000.3, z0=7.5, a=0.05."""
    inj = [Injection(series=0, kind="sine", r0=10000.3, z0=7.5, amp=0.05)]
    return Workload("plain-fdas-1x2^17", 1, 1 << 17, 1, 2.0e-4, 20.0, 2.0, 1, 6.0, inj, noise=noise)


def _pulsar_draws(rng, nsamp, tsamp, zabs_max, amp_lo=0.05, amp_hi=0.5):
    tobs = nsamp * tsamp
    period = math.exp(rng.uniform(math.log(1e-3), math.log(0.5)))   # seconds
    duty = rng.uniform(0.02, 0.10)
    z0 = rng.uniform(-zabs_max, zabs_max)
    amp = math.exp(rng.uniform(math.log(amp_lo), math.log(amp_hi)))
    r0 = tobs / period
    phase0 = rng.uniform(0.0, 1.0)
    return r0, z0, amp, duty, phase0


def config2(nseries: int = 128, nsamp: int = 1 << 18) -> Workload:
    """FAST drift-scan shaped batch: 128 x 2^18 at 0.2 ms; 8 series carry pulse trains."""
    rng = np.random.Generator(np.random.PCG64(seed_for(2, 999)))
    carriers = sorted(rng.choice(nseries, size=min(8, nseries), replace=False).tolist())
    inj = []
    for b in carriers:
        r0, z0, amp, duty, ph = _pulsar_draws(rng, nsamp, 2.0e-4, 150.0)
        inj.append(Injection(series=int(b), kind="pulse", r0=r0, z0=z0, amp=amp, duty=duty, phase0=ph))
    return Workload("fast-batch-128x2^18", 2, nsamp, nseries, 2.0e-4, 200.0, 2.0, 8, 6.0, inj)


def config3(nseries: int = 32, nsamp: int = 1 << 23) -> Workload:
    """PMPS shaped long series: 32 x 2^23 at 250 us; binary-like pulse trains and RFI tones."""
    tsamp = 2.5e-4
    tobs = nsamp * tsamp
    rng = np.random.Generator(np.random.PCG64(seed_for(3, 999)))
    carriers = sorted(rng.choice(nseries, size=min(8, nseries), replace=False).tolist())
    inj = []
    for b in carriers:
        r0, z0, amp, duty, ph = _pulsar_draws(rng, nsamp, tsamp, 200.0)
        inj.append(Injection(series=int(b), kind="pulse", r0=r0, z0=z0, amp=amp, duty=duty, phase0=ph))
    for f_hz, a in ((50.0, 0.3), (100.0, 0.1), (150.0, 0.05)):
        inj.append(Injection(series=-1, kind="tone", r0=f_hz * tobs, z0=0.0, amp=a))
    return Workload("pmps-long-32x2^23", 3, nsamp, nseries, tsamp, 200.0, 2.0, 16, 6.0, inj)


@dataclasses.dataclass
class RaggedWorkload:
    """A batch whose series differ in length, sampling time and searched drift."""
    name: str
    config: int
    nsamp: List[int]
    tsamp: List[float]
    zmax: List[float]
    dz: float
    numharm: int
    sigma: float
    injections: List[Injection]
    noise: bool = True

    @property
    def nseries(self) -> int:
        return len(self.nsamp)

    def offsets(self, series_idx=None) -> np.ndarray:
        """Start of each selected series in the packed buffer (elements)."""
        idx = range(self.nseries) if series_idx is None else series_idx
        n = np.array([self.nsamp[i] for i in idx], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)


def config4(nseries: int = 512, tobs: float = 52.4288, noise: bool = True) -> RaggedWorkload:
    """Uneven batch: 512 series of 2^16..2^20 samples (exponent uniform, so lengths are
    log-uniform) covering the same 52.4288 s, as dedispersion trials downsampled by
    different factors are; zmax per series from {0, 50, 100, 200, 300}; 10 % of the
    series carry a pulse train with |z| <= 0.75 zmax."""
    rng = np.random.Generator(np.random.PCG64(seed_for(4, 999)))
    expo = rng.integers(16, 21, nseries)
    nsamp = [int(1 << int(e)) for e in expo]
    tsamp = [tobs / n for n in nsamp]
    zchoices = np.array([0.0, 50.0, 100.0, 200.0, 300.0])
    zmax = [float(z) for z in zchoices[rng.integers(0, 5, nseries)]]
    carriers = sorted(rng.choice(nseries, size=max(1, nseries // 10), replace=False).tolist())
    inj = []
    for b in carriers:
        ts = tsamp[b]
        period = math.exp(rng.uniform(math.log(max(8 * ts, 1e-3)), math.log(0.5)))
        inj.append(Injection(series=int(b), kind="pulse", r0=tobs / period,
                             z0=rng.uniform(-0.75, 0.75) * zmax[b],
                             amp=math.exp(rng.uniform(math.log(0.05), math.log(0.5))),
                             duty=rng.uniform(0.02, 0.10), phase0=rng.uniform(0.0, 1.0)))
    return RaggedWorkload(f"uneven-{nseries}x2^16..2^20", 4, nsamp, tsamp, zmax, 2.0, 8, 6.0, inj,
                          noise=noise)


def small_ragged(nsamp, tsamp, zmax, dz: float = 2.0, numharm: int = 4, sigma: float = 6.0,
                 config: int = 98, signals: int = 3, amp_range=(0.2, 0.8)) -> RaggedWorkload:
    """A small seeded ragged batch for parity tests (pulse trains in a few series)."""
    rng = np.random.Generator(np.random.PCG64(seed_for(config, 777)))
    nser = len(nsamp)
    inj = []
    for b in sorted(rng.choice(nser, size=min(signals, nser), replace=False).tolist()):
        tobs = nsamp[b] * tsamp[b]
        period = math.exp(rng.uniform(math.log(max(8 * tsamp[b], 2e-3)), math.log(tobs / 40.0)))
        inj.append(Injection(series=int(b), kind="pulse", r0=tobs / period,
                             z0=rng.uniform(-0.75, 0.75) * zmax[b],
                             amp=math.exp(rng.uniform(math.log(amp_range[0]), math.log(amp_range[1]))),
                             duty=rng.uniform(0.02, 0.10), phase0=rng.uniform(0, 1)))
    return RaggedWorkload(f"ragged-{nser}", config, [int(n) for n in nsamp], [float(t) for t in tsamp],
                          [float(z) for z in zmax], dz, numharm, sigma, inj)


def generate_series(wl, b: int) -> np.ndarray:
    """Series b of a ragged workload as float32 [nsamp[b]]."""
    x = _series(wl.nsamp[b], seed_for(wl.config, b), wl.noise)
    for inj in wl.injections:
        if inj.series == b:
            add_pulse(x, inj.r0, inj.z0, inj.amp, inj.duty, inj.phase0)
    return x.astype(np.float32)


def generate_ragged(wl: RaggedWorkload, series_idx=None) -> np.ndarray:
    """The selected series packed back to back (float32), in the order given;
    their starts are wl.offsets(series_idx)."""
    idx = list(range(wl.nseries)) if series_idx is None else list(series_idx)
    out = np.empty(sum(wl.nsamp[i] for i in idx), dtype=np.float32)
    pos = 0
    for i in idx:
        out[pos:pos + wl.nsamp[i]] = generate_series(wl, i)
        pos += wl.nsamp[i]
    return out


def red_noise_batch(nseries: int, nsamp: int, walk_sd: float, config: int = 88) -> np.ndarray:
    """float32 [nseries][nsamp]: white N(0,1) noise plus a random walk with steps of
    sd walk_sd (power falling as 1/f^2: red noise)."""
    out = np.empty((nseries, nsamp), dtype=np.float32)
    for b in range(nseries):
        rng = np.random.Generator(np.random.PCG64(seed_for(config, b)))
        x = rng.standard_normal(nsamp) + np.cumsum(walk_sd * rng.standard_normal(nsamp))
        out[b] = x.astype(np.float32)
    return out


def generate(wl: Workload, series_idx=None) -> np.ndarray:
    """float32 [len(series_idx)][nsamp]; default: the whole batch."""
    if series_idx is None:
        series_idx = list(range(wl.nseries))
    return _render(wl, list(series_idx))


def _render_one(args):
    wl, b = args
    return _render(wl, [b])[0]


def generate_parallel(wl: Workload, series_idx=None, workers: int = 16) -> np.ndarray:
    """generate() with the series drawn in up to `workers` processes (same bytes: each
    series has its own seeded stream). For the long-series batches, whose serial
    generation takes tens of seconds."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    idx = list(range(wl.nseries)) if series_idx is None else list(series_idx)
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    nw = max(1, min(workers, avail, len(idx)))
    if nw == 1:
        return generate(wl, idx)
    out = np.empty((len(idx), wl.nsamp), dtype=np.float32)
    with cf.ProcessPoolExecutor(nw, mp_context=mp.get_context("spawn")) as ex:
        for row, x in enumerate(ex.map(_render_one, [(wl, b) for b in idx])):
            out[row] = x
    return out


def small_batch(nseries: int, nsamp: int, tsamp: float, zmax: float, dz: float, numharm: int,
                sigma: float = 6.0, config: int = 90, signals: int = 2, zabs_max: float = None,
                amp_range=(0.05, 0.5), noise: bool = True) -> Workload:
    """A small seeded batch with pulse trains in a few series, for parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed_for(config, 777)))
    zabs = zmax * 0.75 if zabs_max is None else zabs_max
    inj = []
    for i in range(min(signals, nseries)):
        b = int(rng.integers(0, nseries))
        tobs = nsamp * tsamp
        # keep the fundamental well inside the searched band
        period = math.exp(rng.uniform(math.log(max(8 * tsamp, 2e-3)), math.log(tobs / 40.0)))
        r0 = tobs / period
        inj.append(Injection(series=b, kind="pulse", r0=r0, z0=rng.uniform(-zabs, zabs),
                             amp=math.exp(rng.uniform(math.log(amp_range[0]), math.log(amp_range[1]))),
                             duty=rng.uniform(0.02, 0.10), phase0=rng.uniform(0, 1)))
    return Workload(f"small-{nseries}x{nsamp}", config, nsamp, nseries, tsamp, zmax, dz, numharm,
                    sigma, inj, noise=noise)


# --------------------------------------------------------------------------- filterbank data

# Dedispersion plans of the paper: (DM start, DM step, number of DMs, downsampling
# factor) per range, Table 2 (PMPS) and Table 3 (FAST drift scan).
DDPLAN_PMPS = [(0.0, 0.5, 228, 1), (114.0, 1.0, 152, 2), (266.0, 2.0, 105, 4), (476.0, 5.0, 76, 8),
               (856.0, 10.0, 152, 16), (2376.0, 20.0, 76, 32)]
DDPLAN_FAST = [(0.0, 0.1, 315, 8), (31.5, 0.2, 157, 16), (62.9, 0.5, 153, 32), (139.4, 1.0, 139, 64),
               (278.4, 2.0, 139, 128), (556.4, 3.0, 76, 128)]

# Signal model of dispersion: a pulse emitted at time t arrives in channel c at
# t + K DM f_c^-2 (cold plasma, K in MHz^2 s cm^3/pc); only differences between
# channels matter here, so arrival times are taken relative to the highest channel.
_DISPERSION_K = 4.148808e3


@dataclasses.dataclass
class DispersedPulsar:
    period: float        # s
    dm: float            # pc cm^-3
    amp: float           # peak height per channel, in raw sample units
    duty: float          # FWHM as a fraction of the period
    phase0: float = 0.0  # cycles, at t = 0 in the highest channel


@dataclasses.dataclass
class Filterbank:
    name: str
    nchan: int
    nsamp: int
    tsamp: float
    f0: float            # centre frequency of channel 0 (MHz)
    df: float            # channel spacing (MHz; negative for a descending band)
    pulsars: List[DispersedPulsar]
    plan: list           # DM plan ranges (dm_start, dm_step, ndm, downsamp)
    seed: int
    mean: float = 100.0
    sd: float = 10.0

    def freqs(self) -> np.ndarray:
        return self.f0 + np.arange(self.nchan, dtype=np.float64) * self.df


def fast_filterbank(nsamp: int = 1 << 18) -> Filterbank:
    """FAST drift-scan file shape (Table 1): 200 channels of 0.25 MHz over 290-340 MHz,
    0.2 ms sampling, 2^18 samples (52.4288 s), 8 bits; three dispersed pulsars."""
    psr = [DispersedPulsar(0.08731, 12.3, 0.3, 0.05, 0.1), DispersedPulsar(0.31412, 45.6, 0.5, 0.03, 0.6),
           DispersedPulsar(0.02573, 88.8, 0.25, 0.08, 0.3)]
    return Filterbank("fast-filterbank-200x2^18", 200, nsamp, 2.0e-4, 290.125, 0.25, psr, DDPLAN_FAST,
                      seed_for(6, 0))


def pmps_filterbank(nsamp: int = 1 << 23) -> Filterbank:
    """PMPS file shape (Table 1): 96 channels of 3 MHz over 1231.5-1516.5 MHz (descending),
    250 us sampling, 2^23 samples, 8 bits; two dispersed pulsars."""
    psr = [DispersedPulsar(0.4471, 180.5, 0.1, 0.04, 0.2), DispersedPulsar(0.00412, 33.3, 0.04, 0.10, 0.7)]
    return Filterbank("pmps-filterbank-96x2^23", 96, nsamp, 2.5e-4, 1515.0, -3.0, psr, DDPLAN_PMPS,
                      seed_for(7, 0))


def small_filterbank(nchan: int, nsamp: int, tsamp: float, f0: float, df: float, plan, pulsars=(),
                     config: int = 97) -> Filterbank:
    return Filterbank(f"filterbank-{nchan}x{nsamp}", nchan, nsamp, tsamp, f0, df, list(pulsars), list(plan),
                      seed_for(config, 1))


def generate_filterbank(fb: Filterbank, block: int = 1 << 16) -> np.ndarray:
    """uint8 [nsamp][nchan] (time-major, as filterbank files store it): Gaussian noise of
    the given mean and sd plus von Mises pulse trains delayed per channel by dispersion,
    rounded to integers and clipped to 0..255. Generated in time blocks."""
    rng = np.random.Generator(np.random.PCG64(fb.seed))
    f = fb.freqs()
    fhi = float(np.max(f))
    out = np.empty((fb.nsamp, fb.nchan), dtype=np.uint8)
    for t0 in range(0, fb.nsamp, block):
        n = min(block, fb.nsamp - t0)
        x = fb.mean + fb.sd * rng.standard_normal((n, fb.nchan))
        t = (t0 + np.arange(n, dtype=np.float64))[:, None] * fb.tsamp
        for p in fb.pulsars:
            delay = _DISPERSION_K * p.dm * (1.0 / (f * f) - 1.0 / (fhi * fhi))
            ph = (t - delay[None, :]) / p.period + p.phase0
            kappa = von_mises_kappa(p.duty)
            x += p.amp * np.exp(kappa * (np.cos(2.0 * np.pi * ph) - 1.0))
        out[t0:t0 + n] = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    return out
