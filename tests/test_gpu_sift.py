"""Local-median (red-noise) normalisation on the GPU against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from fdas_check import OracleSeries, assert_candidates_match

pytestmark = pytest.mark.gpu


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.mark.parametrize("N", [64, 1 << 12, 1 << 16])
def test_local_normalisation_matches_oracle(fdas_gpu, N):
    x = synth.red_noise_batch(3, N, 0.05)
    plan = fdas_gpu.Plan(N, 3, 0.0, 2.0, 1, norm="local")
    A, norm = plan.spectrum(_cuda(x))
    A = A.cpu().numpy().astype(np.complex128)
    assert np.all(np.isnan(norm))
    for b in range(3):
        ref, _ = O.deredden(O.spectrum(x[b]))
        pg, po = np.abs(A[b]) ** 2, np.abs(ref) ** 2
        err = np.abs(pg - po) / np.maximum(po, 1.0)
        assert err.max() <= 1e-4, (b, float(err.max()), int(np.argmax(err)))
        assert A[b][0] == 0 and A[b][-1] == 0


def test_local_normalisation_search_matches_oracle(fdas_gpu):
    B, N, ts, zmax, dz, nh = 3, 1 << 14, 1e-3, 20.0, 2.0, 4
    wl = synth.small_batch(B, N, ts, zmax, dz, nh, sigma=5.0, config=91, signals=B, amp_range=(0.4, 0.9))
    x = synth.generate(wl) + synth.red_noise_batch(B, N, 0.05, config=89)
    plan = fdas_gpu.Plan(N, B, zmax, dz, nh, norm="local")
    g = plan.search(_cuda(x), ts, sigma=5.0, cap=1 << 18)
    oracles = {b: OracleSeries(x[b], ts, zmax, dz, nh, norm="local", method="fft") for b in range(B)}
    common, _ = assert_candidates_match(g, oracles, 5.0)
    assert common >= 3
    # the global median leaves the red noise in: many more low-frequency candidates
    g2 = fdas_gpu.Plan(N, B, zmax, dz, nh).search(_cuda(x), ts, sigma=5.0, cap=1 << 18)
    assert len(g2) > len(g)


def test_local_normalisation_ragged_graph_equals_eager(fdas_gpu):
    n = [1 << 12, 1 << 13, 1 << 12, 1 << 14]
    t = [1e-3, 1e-3, 2e-3, 5e-4]
    z = [10.0, 0.0, 20.0, 10.0]
    wl = synth.small_ragged(n, t, z, 2.0, 4, 4.0, config=87, signals=3, amp_range=(0.5, 1.0))
    buf = synth.generate_ragged(wl)
    red = np.concatenate([synth.red_noise_batch(1, k, 0.05, config=86 + i)[0] for i, k in enumerate(n)])
    d = _cuda(buf + red)
    offs = wl.offsets()
    eager = fdas_gpu.Plan(max(n), 4, 20.0, 2.0, 4, norm="local")
    graph = fdas_gpu.Plan(max(n), 4, 20.0, 2.0, 4, norm="local", graph=1)
    for sigma in (4.0, 5.0):
        a = eager.search_ragged(d, offs, n, t, z, sigma=sigma, cap=1 << 18)
        b = graph.search_ragged(d, offs, n, t, z, sigma=sigma, cap=1 << 18)
        assert np.array_equal(a, b)
