"""Dedispersion kernels against the exact integer oracle (bit for bit), and the
dedispersed FAST-shaped file searched as one ragged batch."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _u8(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _check_plan(F, fb, x, plan_ranges):
    plan = F.Plan(1 << 12, 1, 0.0, 2.0, 1)
    _, series = plan.dedisperse(_u8(x), fb.tsamp, fb.f0, fb.df, plan_ranges)
    ref = O.dedisperse_plan(x, fb.freqs(), fb.tsamp, plan_ranges)
    for r, (g, o) in enumerate(zip(series, ref)):
        g = g.cpu().numpy()
        assert g.shape == o.shape, r
        assert np.array_equal(g.astype(np.int64), o), (r, np.argwhere(g.astype(np.int64) != o)[:5])
    return series


@pytest.mark.parametrize("nchan,f0,df", [(37, 420.0, -1.5), (64, 300.0, 0.5), (5, 1500.0, -30.0)])
def test_plan_ranges_bit_exact(fdas_gpu, nchan, f0, df):
    # factors 1, 2, 4 (rows derived from the previous range), 4 again (same rows),
    # 3 (from the file), 6 (from the factor-3 rows)
    ranges = [(0.0, 0.7, 21, 1), (14.7, 1.3, 18, 2), (38.1, 2.0, 9, 4), (56.1, 3.5, 5, 4), (73.6, 4.0, 7, 3),
              (101.6, 9.0, 4, 6)]
    fb = synth.small_filterbank(nchan, 12288, 3e-4, f0, df, ranges,
                                [synth.DispersedPulsar(0.0377, 21.0, 6.0, 0.05, 0.2)], config=95 + nchan)
    x = synth.generate_filterbank(fb)
    _check_plan(fdas_gpu, fb, x, ranges)


def test_wide_delay_spreads_use_smaller_dm_groups(fdas_gpu):
    # low frequencies and coarse DM steps: delays differ by thousands of samples
    # between neighbouring trials, beyond what a 16-DM LDS stage holds
    ranges = [(0.0, 40.0, 19, 1), (0.0, 0.01, 33, 2)]
    fb = synth.small_filterbank(9, 1 << 14, 1e-4, 100.0, 2.0, ranges, config=93)
    x = synth.generate_filterbank(fb)
    _check_plan(fdas_gpu, fb, x, ranges)


def test_invalid_arguments(fdas_gpu):
    import torch
    F = fdas_gpu
    plan = F.Plan(1 << 12, 1, 0.0, 2.0, 1)
    x = torch.zeros((1000, 8), dtype=torch.uint8, device="cuda")
    for ranges in ([(0.0, 1.0, 4, 3)], [(-1.0, 1.0, 4, 1)], [(0.0, -1.0, 4, 1)], [(0.0, 1.0, 0, 1)]):
        with pytest.raises(F.FdasError) as e:
            plan.dedisperse(x, 1e-3, 400.0, -1.0, ranges)
        assert e.value.status == F.FDAS_E_INVAL
    with pytest.raises(F.FdasError):
        plan.dedisperse(x, 1e-3, 4.0, -1.0, [(0.0, 1.0, 4, 1)])         # last channel below 0 MHz
    # output capacity is checked by the C ABI
    lib = F.load()
    rg = np.zeros(1, dtype=F.DM_RANGE_DTYPE)
    rg[0] = (0.0, 1.0, 4, 1)
    out = torch.empty(3999, dtype=torch.float32, device="cuda")
    st = lib.fdas_dedisperse(plan.handle, ctypes.c_void_p(x.data_ptr()), 1000, 8, 1e-3, 400.0, -1.0,
                             rg.ctypes.data_as(ctypes.c_void_p), 1, ctypes.c_void_p(out.data_ptr()), out.numel(),
                             None)
    assert st == F.FDAS_E_INVAL


@pytest.fixture(scope="module")
def fast_file(fdas_gpu):
    fb = synth.fast_filterbank()
    x = synth.generate_filterbank(fb)
    plan = fdas_gpu.Plan(1 << 15, 1024, 50.0, 2.0, 8)
    buf, series = plan.dedisperse(_u8(x), fb.tsamp, fb.f0, fb.df, fb.plan)
    return fb, x, plan, buf, series


def test_fast_file_with_table3_plan_bit_exact(fast_file):
    fb, x, _, _, series = fast_file
    ref = O.dedisperse_plan(x, fb.freqs(), fb.tsamp, fb.plan)
    for r, (g, o) in enumerate(zip(series, ref)):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), o), r


def test_dedispersed_batch_search_finds_the_pulsars(fast_file):
    """The packed output is a ragged batch: one fdas_search_ragged call over all 979 trials."""
    fb, _, plan, buf, series = fast_file
    offs, ns, ts, dms = [], [], [], []
    o = 0
    for (a, s, n, d), sr in zip(fb.plan, series):
        for i in range(n):
            offs.append(o + i * sr.shape[1])
            ns.append(sr.shape[1])
            ts.append(fb.tsamp * d)
            dms.append(a + i * s)
        o += n * sr.shape[1]
    cands = plan.search_ragged(buf, offs, ns, ts, 0.0, dz=2.0, numharm=8, sigma=8.0, cap=1 << 20)
    T = (np.array(ns) * np.array(ts))[cands["series"]]
    dm_of = np.array(dms)[cands["series"]]
    for p in fb.pulsars:
        near = np.abs(cands["f_hz"] - 1.0 / p.period) <= 2.0 / T
        assert near.any(), p
        assert np.min(np.abs(dm_of[near] - p.dm)) <= 3.0, (p, np.sort(dm_of[near])[:5])


def test_sifted_dedispersed_search_keeps_each_pulsar_once(fast_file, fdas_gpu):
    """Sifting the 979-trial candidate list: every pulsar survives as a strong entry that
    stands for its detections over many trial DMs around its own DM."""
    fb, _, plan, buf, series = fast_file
    offs, ns, ts, dms = [], [], [], []
    o = 0
    for (a, s, n, d), sr in zip(fb.plan, series):
        for i in range(n):
            offs.append(o + i * sr.shape[1])
            ns.append(sr.shape[1])
            ts.append(fb.tsamp * d)
            dms.append(a + i * s)
        o += n * sr.shape[1]
    cands = plan.search_ragged(buf, offs, ns, ts, 0.0, dz=2.0, numharm=8, sigma=7.0, cap=1 << 20)
    sifted = fdas_gpu.sift(cands)
    assert 0 < len(sifted) < len(cands) / 5
    for p in fb.pulsars:
        f = 1.0 / p.period
        rows = [r for r in sifted if abs(cands[r["index"]]["f_hz"] - f) <= 2.0 / 52.4288]
        assert len(rows) == 1, (p, len(rows))
        r = rows[0]
        assert r["hits"] >= 5
        assert dms[r["series_lo"]] <= p.dm + 3.0 and dms[r["series_hi"]] >= p.dm - 3.0
