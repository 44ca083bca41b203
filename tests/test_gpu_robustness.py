"""Failure handling on the device path: allocation failures injected through the
plan option fail_alloc (the n-th allocation made for a plan fails as if memory
were exhausted) return FDAS_E_NOMEM, leave no plan behind at creation, and leave
a plan that searches correctly afterwards (also with graph replay, whose
captured buffers a failed regrowth frees)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _batch():
    B, N, ts = 3, 1 << 13, 1e-3
    wl = synth.small_batch(B, N, ts, 20.0, 2.0, 4, config=95, signals=3, amp_range=(0.3, 0.8))
    return B, N, ts, _cuda(synth.generate(wl))


def _creation_allocations(fdas, B, N, **kw):
    """Fail each allocation of plan creation in turn; returns how many there are."""
    k = 1
    while True:
        try:
            plan = fdas.Plan(N, B, 20.0, 2.0, 4, fail_alloc=k, **kw)
        except fdas.FdasError as e:
            assert e.status == fdas.FDAS_E_NOMEM, e
            k += 1
            assert k < 100
            continue
        plan.close()
        return k - 1


def test_injected_failures_at_plan_creation(fdas_gpu):
    B, N, _, _ = _batch()
    n = _creation_allocations(fdas_gpu, B, N)
    assert n >= 20      # bank, spectra, FFT scratch, plane, maxima, records, staging, ...


@pytest.mark.parametrize("graph", [0, 1])
def test_plan_usable_after_each_injected_failure(fdas_gpu, graph):
    """Every allocation a sequence of searches makes after plan creation (row-block
    tables, record regrowth beyond max_candidates, host staging, a second template
    bank) fails in turn: the call that hits it returns FDAS_E_NOMEM, the same call
    then succeeds, and every result equals that of a plan without failures."""
    B, N, ts, x = _batch()
    steps = [dict(sigma=9.0), dict(sigma=3.0, cap=1 << 18), dict(zmax=10.0, sigma=6.0),
             dict(sigma=3.0, cap=1 << 18), dict(sigma=9.0)]
    ref = fdas_gpu.Plan(N, B, 20.0, 2.0, 4, max_candidates=64)
    want = [ref.search(x, ts, **kw) for kw in steps]
    ref.close()
    assert len(want[1]) > 64 and len(want[0]) <= 64
    n = _creation_allocations(fdas_gpu, B, N, graph=graph, max_candidates=64)
    hits = 0
    for k in range(n + 1, n + 40):
        plan = fdas_gpu.Plan(N, B, 20.0, 2.0, 4, fail_alloc=k, graph=graph, max_candidates=64)
        failed = False
        for kw, w in zip(steps, want):
            try:
                got = plan.search(x, ts, **kw)
            except fdas_gpu.FdasError as e:
                assert e.status == fdas_gpu.FDAS_E_NOMEM and "injected" in str(e), e
                assert not failed
                failed = True
                got = plan.search(x, ts, **kw)
            assert np.array_equal(got, w), (k, kw)
        plan.close()
        if not failed:
            break
        hits += 1
    assert hits >= 4, hits      # row tables, records, staging, second bank at least
