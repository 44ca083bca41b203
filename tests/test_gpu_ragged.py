"""Ragged batches: series of different lengths, sampling times and drift ranges
searched in one call, against the FP64 oracle series by series, against the
plain per-series calls (bit for bit: same kernels, same launch parameters),
under graph replay and with the autotuner.
"""
import numpy as np
import pytest

import synth
from fdas_check import OracleSeries, assert_candidates_match

pytestmark = pytest.mark.gpu

# (nsamp, tsamp, zmax): groups by (nsamp, lowest bin, zmax); series 1 and 6
# share a group, series 1 and 3 differ only in tsamp (another lowest bin),
# series 6 and 7 share nsamp, band and zmax but not tsamp (same group, other T),
# series 5 is shorter than one correlation segment.
RAGGED = [
    (1 << 12, 1e-3, 0.0),
    (1 << 13, 1e-3, 10.0),
    (1 << 14, 5e-4, 20.0),
    (1 << 13, 2e-3, 10.0),
    (1 << 12, 1e-3, 40.0),
    (1 << 9, 1e-3, 10.0),
    (1 << 13, 1e-3, 10.0),
    (1 << 13, 1.01e-3, 10.0),
]
DZ, NH, SIGMA = 2.0, 4, 4.0


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def ragged():
    n, t, z = zip(*RAGGED)
    wl = synth.small_ragged(n, t, z, DZ, NH, SIGMA, config=98, signals=4, amp_range=(0.5, 1.5))
    buf = synth.generate_ragged(wl)
    return wl, buf, wl.offsets()


def _plan(F, wl, **kw):
    return F.Plan(max(wl.nsamp), wl.nseries, max(wl.zmax), wl.dz, wl.numharm, **kw)


def _series(wl, buf, offs, i):
    return buf[offs[i]:offs[i] + wl.nsamp[i]]


def _check_vs_oracle(cands, wl, buf, offs):
    common = 0
    for i in range(wl.nseries):
        orc = OracleSeries(_series(wl, buf, offs, i), wl.tsamp[i], wl.zmax[i], wl.dz, wl.numharm,
                           method="fft")
        c, _ = assert_candidates_match(cands[cands["series"] == i], {i: orc}, wl.sigma)
        common += c
    return common


def test_ragged_matches_oracle_per_series(fdas_gpu, ragged):
    wl, buf, offs = ragged
    plan = _plan(fdas_gpu, wl)
    g = plan.search_ragged(_cuda(buf), offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    keys = [(int(c["series"]), int(c["harm"]), int(c["r_idx"])) for c in g]
    assert keys == sorted(keys)
    assert _check_vs_oracle(g, wl, buf, offs) >= 20
    # units use each series' own observation length
    T = np.array([wl.nsamp[i] * wl.tsamp[i] for i in range(wl.nseries)])
    assert np.allclose(g["f_hz"], g["r_fund"] / T[g["series"]], rtol=1e-15)
    assert np.allclose(g["fdot_hz_s"], g["z_fund"] / T[g["series"]] ** 2, rtol=1e-15)


# lengths whose halves are products of powers of 2, 3 and 5 (4374: 3^7, in one
# workgroup; 15360, 12000 and 9720 in one workgroup or four-step)
RAGGED_SMOOTH = [(12000, 1e-3, 20.0), (15360, 1e-3, 10.0), (12000, 1e-3, 0.0), (9720, 2e-3, 20.0),
                 (4374, 1e-3, 10.0), (40000, 5e-4, 20.0)]


def test_ragged_5smooth_lengths_match_oracle(fdas_gpu):
    n, t, z = zip(*RAGGED_SMOOTH)
    wl = synth.small_ragged(n, t, z, DZ, NH, SIGMA, config=84, signals=4, amp_range=(0.5, 1.5))
    buf = synth.generate_ragged(wl)
    offs = wl.offsets()
    plan = _plan(fdas_gpu, wl, graph=1)
    d = _cuda(buf)
    g = plan.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    assert _check_vs_oracle(g, wl, buf, offs) >= 10
    again = plan.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)   # replay
    assert np.array_equal(g, again)


def test_ragged_equals_per_series_calls(fdas_gpu, ragged):
    wl, buf, offs = ragged
    plan = _plan(fdas_gpu, wl)
    g = plan.search_ragged(_cuda(buf), offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    for i in range(wl.nseries):
        one = plan.search(_cuda(_series(wl, buf, offs, i)[None]), wl.tsamp[i], zmax=wl.zmax[i],
                          sigma=wl.sigma, cap=1 << 18)
        one["series"] = i
        assert np.array_equal(g[g["series"] == i], one), i


def test_ragged_waves_in_small_workspace(fdas_gpu, ragged):
    """A workspace of two of the largest planes splits the batch into several
    waves (groups into chunks); the merged harmonic-sum launches of each wave
    give the records of the one-wave search, eagerly and under graph replay."""
    wl, buf, offs = ragged
    d = _cuda(buf)
    ref = _plan(fdas_gpu, wl).search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    nz = 2 * int(round(max(wl.zmax) / wl.dz)) + 1
    pitch = -(-max(wl.nsamp) // 64) * 64
    for graph in (0, 1):
        small = _plan(fdas_gpu, wl, max_workspace_bytes=2 * nz * pitch * 4, graph=graph)
        assert small.info()["chunk_series"] == 2
        for _ in range(2):
            g = small.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
            assert np.array_equal(g, ref), graph


def test_ragged_series_order_and_offsets_are_free(fdas_gpu, ragged):
    """A permuted packing with gaps gives the same records, relabelled."""
    wl, buf, offs = ragged
    plan = _plan(fdas_gpu, wl)
    ref = plan.search_ragged(_cuda(buf), offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    perm = np.random.default_rng(3).permutation(wl.nseries)
    gap = 6
    new_offs = np.zeros(wl.nseries, np.int64)
    parts, pos = [], 0
    for j, i in enumerate(perm):
        parts.append(np.full(gap, 1e3, np.float32))      # junk between series is never read
        pos += gap
        new_offs[j] = pos
        parts.append(_series(wl, buf, offs, i))
        pos += wl.nsamp[i]
    buf2 = np.concatenate(parts)
    g = plan.search_ragged(_cuda(buf2), new_offs, [wl.nsamp[i] for i in perm], [wl.tsamp[i] for i in perm],
                           [wl.zmax[i] for i in perm], sigma=wl.sigma, cap=1 << 18)
    for j, i in enumerate(perm):
        a = ref[ref["series"] == i].copy()
        b = g[g["series"] == j].copy()
        a["series"] = 0
        b["series"] = 0
        assert np.array_equal(a, b), (i, j)


def test_graph_replay_matches_eager(fdas_gpu, ragged):
    import torch
    wl, buf, offs = ragged
    eager = _plan(fdas_gpu, wl)
    graph = _plan(fdas_gpu, wl, graph=1)
    d = _cuda(buf)
    other = np.random.default_rng(11).standard_normal(buf.shape).astype(np.float32)
    runs = [(buf, 5.0), (buf, 6.0), (other, 5.0), (buf, 5.0)]
    for data, sigma in runs:
        d.copy_(torch.from_numpy(data))
        want = eager.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=sigma, cap=1 << 18)
        torch.cuda.synchronize()
        got = graph.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=sigma, cap=1 << 18)
        assert np.array_equal(want, got), sigma
    # homogeneous searches replay as well
    x = _cuda(np.stack([_series(wl, buf, offs, i) for i in (1, 3, 6)]))
    for sigma in (4.0, 5.0, 4.0):
        want = eager.search(x, 1e-3, zmax=10.0, sigma=sigma, cap=1 << 18)
        got = graph.search(x, 1e-3, zmax=10.0, sigma=sigma, cap=1 << 18)
        assert np.array_equal(want, got)


def test_autotune_results_and_tuning_roundtrip(fdas_gpu, ragged):
    F = fdas_gpu
    wl, buf, offs = ragged
    d = _cuda(buf)
    tuned = _plan(F, wl, autotune=1)
    g = tuned.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma, cap=1 << 18)
    assert _check_vs_oracle(g, wl, buf, offs) >= 20
    text = tuned.tuning()
    shapes = {(n, int(round(z / wl.dz))) for n, z in zip(wl.nsamp, wl.zmax)}
    lines = [l.split() for l in text.strip().splitlines()]
    assert {(int(l[0]), int(l[1])) for l in lines} == shapes
    for l in lines:
        assert int(l[2]) == wl.numharm and int(l[3]) in (512, 1024, 2048, 4096) and int(l[5]) in (0, 1)
    # a plan given the same tuning reproduces the records bit for bit
    other = _plan(F, wl)
    other.load_tuning(text)
    assert np.array_equal(g, other.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma,
                                                 cap=1 << 18))
    # a second search on the tuned plan does not re-tune and gives the same records
    assert np.array_equal(g, tuned.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=wl.sigma,
                                                 cap=1 << 18))
    assert tuned.tuning() == text
    for bad in ("65536 10 8 1000 6 0\n", "65536 10 8 1024 6\n", "x y z\n", "4096 5 3 1024 6 0\n"):
        with pytest.raises(F.FdasError) as e:
            other.load_tuning(bad)
        assert e.value.status == F.FDAS_E_INVAL


def test_ragged_truncation_keeps_sorted_prefix(fdas_gpu, ragged):
    wl, buf, offs = ragged
    plan = _plan(fdas_gpu, wl, max_candidates=16)
    d = _cuda(buf)
    full = plan.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=3.0, cap=1 << 18)
    assert len(full) > 40
    part, total = plan.search_ragged(d, offs, wl.nsamp, wl.tsamp, wl.zmax, sigma=3.0, cap=25,
                                     allow_trunc=True)
    assert total == len(full)
    assert np.array_equal(part, full[:25])


def test_ragged_invalid_arguments(fdas_gpu, ragged):
    F = fdas_gpu
    wl, buf, offs = ragged
    plan = _plan(F, wl)
    d = _cuda(buf)
    n, t, z = list(wl.nsamp), list(wl.tsamp), list(wl.zmax)

    def expect(status, offs_=offs, n_=n, t_=t, z_=z, **kw):
        with pytest.raises(F.FdasError) as e:
            plan.search_ragged(d, offs_, n_, t_, z_, **kw)
        assert e.value.status == status

    o = offs.copy()
    o[2] += 1
    expect(F.FDAS_E_INVAL, offs_=o)                           # odd offset
    expect(F.FDAS_E_INVAL, z_=[11.0] + z[1:])                  # zmax not a multiple of dz
    expect(F.FDAS_E_INVAL, t_=[0.0] + t[1:])
    expect(F.FDAS_E_INVAL, numharm=8)                          # above the plan's numharm
    expect(F.FDAS_E_UNSUPPORTED, n_=[n[0] - 16] + n[1:])       # N/2 = 2040 has the prime factor 17
    with pytest.raises(ValueError):
        plan.search_ragged(d, offs + 8, n, t, z)               # last series past the buffer
    big = F.Plan(1 << 12, 2, 10.0, 2.0, 4)
    with pytest.raises(F.FdasError) as e:
        big.search_ragged(d, offs[:2], n[:2], t[:2], [0.0, 10.0])   # nsamp above max_nsamp
    assert e.value.status == F.FDAS_E_INVAL
    # the plan still works after rejected calls
    assert plan.search_ragged(d, offs, n, t, z, sigma=6.0) is not None
