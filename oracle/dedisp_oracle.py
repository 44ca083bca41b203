"""Plain reference of incoherent dedispersion (integer arithmetic, exact).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 2, step 2 of the paper dedisperses the filterbank data into time
series at many trial DMs (prepdata / prepsubband), with the DM plans of
Tables 2-3 (ranges of trial DMs, each with its own downsampling factor). The
paper does not define the arithmetic; the reading adopted here:

  * cold-plasma delay of channel c (centre frequency f_c, MHz) relative to the
    highest channel frequency f_hi, at dispersion measure DM (pc cm^-3):
        t_c = KDM * DM * (f_c^-2 - f_hi^-2) seconds, KDM = 4.148808e3 MHz^2 s / (pc cm^-3);
  * a range with downsampling factor D first sums D consecutive samples of each
    channel (boxcar): y_c[j] = sum_{d<D} x_c[j D + d], j < nsamp / D;
  * the delay in downsampled samples is the nearest integer, computed in FP64 as
        delta_c = floor(KDM * DM * (f_c^-2 - f_hi^-2) / (D * tsamp) + 1/2);
  * the dedispersed series is out[j] = sum_c y_c[j + delta_c], j < nsamp / D,
    with y_c read past its end as p_c = floor((D sum_t x_c[t] + nsamp/2) / nsamp),
    the channel's boxcar mean rounded to an integer (so that late samples of
    high-DM trials keep the series level, to within half a unit per channel,
    instead of stepping down).

With 8-bit samples every sum is an integer below 2^24, so the result is exact
in float32 as well as in the int64 used here.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = ["KDM", "channel_freqs", "dm_delays", "downsample", "channel_pad", "dedisperse",
           "dedisperse_plan", "range_dms"]

KDM = 4.148808e3        # MHz^2 s / (pc cm^-3)


def channel_freqs(nchan: int, f0_mhz: float, df_mhz: float) -> np.ndarray:
    """Centre frequency of channel c: f0 + c df (df may be negative)."""
    return float(f0_mhz) + np.arange(nchan, dtype=np.float64) * float(df_mhz)


def dm_delays(dm: float, freqs: np.ndarray, tsamp: float, down: int) -> np.ndarray:
    """delta_c = floor(KDM DM (f_c^-2 - f_hi^-2) / (D tsamp) + 1/2) for every channel (int64)."""
    f = np.asarray(freqs, dtype=np.float64)
    fhi = float(np.max(f))
    x = KDM * float(dm) * (1.0 / (f * f) - 1.0 / (fhi * fhi)) / (float(down) * float(tsamp))
    return np.floor(x + 0.5).astype(np.int64)


def downsample(x: np.ndarray, down: int) -> np.ndarray:
    """Boxcar sums of D consecutive samples; x: [nsamp][nchan] -> y: [nchan][nsamp/D] (int64)."""
    ns, nc = x.shape
    if ns % down:
        raise ValueError("nsamp must be a multiple of the downsampling factor")
    return x.astype(np.int64).reshape(ns // down, down, nc).sum(axis=1).T.copy()


def channel_pad(x: np.ndarray, down: int) -> np.ndarray:
    """p_c = floor((D sum_t x[t][c] + nsamp // 2) / nsamp): each channel's boxcar mean
    over D samples, rounded (int64)."""
    ns = x.shape[0]
    return (int(down) * x.astype(np.int64).sum(axis=0) + ns // 2) // ns


def dedisperse(x: np.ndarray, freqs: np.ndarray, tsamp: float, dms: Sequence[float], down: int) -> np.ndarray:
    """out[i][j] = sum_c y_c[j + delta_c(dms[i])], y_c read as p_c past its end;
    int64 [len(dms)][nsamp/D]."""
    y = downsample(x, down)
    pad = channel_pad(x, down)
    nc, n = y.shape
    out = np.zeros((len(dms), n), dtype=np.int64)
    for i, dm in enumerate(dms):
        d = dm_delays(dm, freqs, tsamp, down)
        for c in range(nc):
            k = min(int(d[c]), n)
            out[i, :n - k] += y[c, k:]
            out[i, n - k:] += pad[c]
    return out


def range_dms(dm_start: float, dm_step: float, ndm: int) -> List[float]:
    """Trial DMs of one plan range: dm_start + i dm_step, i < ndm."""
    return [float(dm_start) + i * float(dm_step) for i in range(int(ndm))]


def dedisperse_plan(x: np.ndarray, freqs: np.ndarray, tsamp: float,
                    ranges: Sequence[Tuple[float, float, int, int]]) -> List[np.ndarray]:
    """Every range (dm_start, dm_step, ndm, D) of a DM plan, in order."""
    return [dedisperse(x, freqs, tsamp, range_dms(a, s, n), D) for a, s, n, D in ranges]
