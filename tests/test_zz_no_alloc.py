"""The entry point that allocates nothing (fdas_spectrum_noalloc) against
fdas_spectrum on a plan, through the C ABI: the same spectra bit for bit and
the same median norms, on two calls in a row (the second smaller, so that the
fixed scratch holds the first call's contents), and its size limit."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def test_noalloc_spectrum_equals_plan_spectrum_on_consecutive_calls(fdas_gpu):
    import torch
    cases = [(6, 1 << 18, 11), (3, 1 << 12, 12)]      # second call smaller than the first
    got = []
    for B, N, cfg in cases:
        x = _cuda(synth.red_noise_batch(B, N, 0.02, config=cfg))
        A, norm = fdas_gpu.spectrum_noalloc(x)
        torch.cuda.synchronize()
        got.append((x, A.clone(), norm.copy()))
    for (B, N, _), (x, A, norm) in zip(cases, got):
        ref_A, ref_norm = fdas_gpu.Plan(N, B, 0.0, 2.0, 1).spectrum(x)
        assert A.shape == ref_A.shape
        assert torch.equal(torch.view_as_real(A), torch.view_as_real(ref_A)), (B, N)
        assert np.array_equal(norm, ref_norm), (B, N, norm, ref_norm)
        assert np.all(norm > 0)


def test_noalloc_spectrum_on_a_side_stream_and_limits(fdas_gpu):
    import torch
    lib = fdas_gpu.load()
    B, N = 2, 1 << 14
    x = _cuda(synth.red_noise_batch(B, N, 0.02, config=13))
    ref_A, ref_norm = fdas_gpu.Plan(N, B, 0.0, 2.0, 1).spectrum(x)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A, norm = fdas_gpu.spectrum_noalloc(x, stream=s)
    s.synchronize()
    assert torch.equal(torch.view_as_real(A), torch.view_as_real(ref_A))
    assert np.array_equal(norm, ref_norm)
    out = torch.empty((B, N // 2 + 1, 2), dtype=torch.float32, device="cuda")
    P = ctypes.c_void_p
    # beyond the fixed scratch: 2 buffers of nseries * N/2 complex values > 64 MiB
    big = lib.fdas_spectrum_noalloc(P(x.data_ptr()), 1 << 24, 1, P(out.data_ptr()), None, None)
    assert big == fdas_gpu.FDAS_E_INVAL
    # nsamp / 2 = 7 * 1024 has a prime factor above 5
    assert lib.fdas_spectrum_noalloc(P(x.data_ptr()), 14 * 1024, 1, P(out.data_ptr()), None, None) == \
        fdas_gpu.FDAS_E_UNSUPPORTED
    assert lib.fdas_spectrum_noalloc(None, N, B, P(out.data_ptr()), None, None) == fdas_gpu.FDAS_E_INVAL
    assert lib.fdas_spectrum_noalloc(P(x.data_ptr()), N, 0, P(out.data_ptr()), None, None) == fdas_gpu.FDAS_E_INVAL
    # nothing launched by the rejected calls: the earlier result is intact
    assert torch.equal(torch.view_as_real(A), torch.view_as_real(ref_A))
