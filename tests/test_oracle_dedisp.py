"""Pins of the dedispersion oracle: the published dispersion constant, brute force
on tiny inputs, DM 0 as the total-power series, hierarchical downsampling, and
a dispersed pulse train that lines up only at its own trial DM."""
import numpy as np
import pytest

import oracle as O
import synth


def test_delay_constant_matches_the_published_value():
    # 4.148808 ms delay for DM 1 pc cm^-3 at 1 GHz relative to infinite frequency
    f = np.array([1000.0, 1e12])
    assert O.KDM * 1.0 * (1 / 1000.0 ** 2 - 1 / 1e24) == pytest.approx(4.148808e-3, rel=1e-12)
    # FAST band edges at the plan's largest DM: about 10.48 s across 290-340 MHz
    fb = synth.fast_filterbank()
    fr = fb.freqs()
    d = O.dm_delays(784.4, fr, fb.tsamp, 128)
    assert d[0] == int(np.floor(4148.808 * 784.4 * (1 / 290.125 ** 2 - 1 / 339.875 ** 2) / (128 * 2e-4) + 0.5))
    assert 400 < d[0] < 420 and d[-1] == 0 and np.all(np.diff(d) <= 0)


def test_brute_force_on_tiny_input():
    rng = np.random.default_rng(1)
    nsamp, nchan, D = 48, 5, 2
    x = rng.integers(0, 256, (nsamp, nchan)).astype(np.uint8)
    fr = np.array([400.0, 380.0, 360.0, 340.0, 320.0])      # descending band
    ts = 1e-3
    dms = [0.0, 3.0, 17.5]
    got = O.dedisperse(x, fr, ts, dms, D)
    n = nsamp // D
    for i, dm in enumerate(dms):
        for j in range(n):
            s = 0
            for c in range(nchan):
                delay = int(np.floor(4.148808e3 * dm * (1 / fr[c] ** 2 - 1 / 400.0 ** 2) / (D * ts) + 0.5))
                jj = j + delay
                if jj < n:
                    for d in range(D):
                        s += int(x[jj * D + d, c])
                else:                                   # past the end: the rounded boxcar mean
                    tot = sum(int(v) for v in x[:, c])
                    s += (2 * D * tot + nsamp) // (2 * nsamp)
            assert got[i, j] == s, (i, j)


def test_zero_dm_is_the_total_power_series():
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, (256, 7)).astype(np.uint8)
    fr = O.channel_freqs(7, 300.0, 2.0)
    out = O.dedisperse(x, fr, 1e-4, [0.0], 4)
    assert np.array_equal(out[0], x.astype(np.int64).reshape(64, 4, 7).sum(axis=(1, 2)))


def test_constant_channels_give_constant_series_at_any_dm():
    # a channel that holds one value everywhere reads the same value past its end,
    # so every trial DM sees the same flat series
    x = np.tile(np.arange(7, dtype=np.uint8) * 30 + 3, (512, 1))
    fr = O.channel_freqs(7, 300.0, 5.0)
    out = O.dedisperse(x, fr, 1e-3, [0.0, 50.0, 400.0], 4)
    assert np.all(out == 4 * int(x[0].astype(np.int64).sum()))


def test_downsampling_is_hierarchical():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (512, 6)).astype(np.uint8)
    y2, y8 = O.downsample(x, 2), O.downsample(x, 8)
    assert np.array_equal(y8, y2.reshape(6, 64, 4).sum(axis=2))


def test_dispersed_pulse_train_lines_up_at_its_dm():
    # trial step 0.25: the residual smearing across the band (<= 59 samples per unit DM
    # here) stays below the 26-sample pulse width at the nearest trial
    fb = synth.small_filterbank(64, 1 << 14, 5e-4, 400.0, -2.0, [(0.0, 0.25, 200, 1)],
                                [synth.DispersedPulsar(1.3, 37.1, 20.0, 0.01, 0.3)])
    fb.sd = 2.0
    x = synth.generate_filterbank(fb)
    dms = O.range_dms(0.0, 0.25, 200)
    out = O.dedisperse(x, fb.freqs(), fb.tsamp, dms, 1)
    peak = out.max(axis=1) - np.median(out, axis=1)
    best = int(np.argmax(peak))
    assert abs(dms[best] - 37.1) <= 0.25, (dms[best], peak[best])
    assert peak[best] > 0.8 * 64 * 20.0            # channels add coherently at the right DM
    assert peak[0] < 0.5 * peak[best]
