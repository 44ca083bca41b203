"""Host-side checks of the C ABI library (no device work).

The library must load, export every symbol the public header declares, and
its host FP64 pieces (response taps, thresholds, significance, geometry)
must agree with the oracle.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    import paper_1912_12807_amd as fdas
    if not os.path.exists(fdas.LIB_PATH):
        from paper_1912_12807_amd import build
        build.build()
    fdas.load()
    return fdas


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "fdas.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fdas_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(F):
    syms = declared_symbols()
    assert len(syms) >= 15
    lib = F.load()       # the library the binding loaded (a sanitized build under test_sanitize_cpu)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(F.EXPORTED)


def test_host_template_taps_match_oracle(F):
    for z in (0.0, 2.0, -2.0, 7.5, -20.0, 150.0, 200.0, -300.0, 0.0004):
        for p in (0, 1):
            for K in (8, 16):
                d0, t = F.template_taps(z, p, K)
                d, to = O.template(z, p, K)
                assert d0 == d[0] and len(t) == len(to)
                assert np.max(np.abs(t - to)) < 1e-11, (z, p, K)


def test_host_thresholds_and_sigma_match_oracle(F):
    for H in (1, 2, 4, 8, 16, 32):
        for s in (3.0, 6.0, 9.0):
            assert F.threshold(H, s) == pytest.approx(O.threshold(H, s), rel=1e-12)
        # powers above the noise mean (the inverse is ill-conditioned where Q -> 1)
        for pw in (H + 5.0, 2.0 * H + 20.0, 300.0, 5000.0):
            assert F.sigma_of(H, pw) == pytest.approx(O.candidate_sigma(H, pw), rel=1e-9, abs=1e-9)
        # dense over the range candidates take (the Newton stopping rule included)
        for pw in np.geomspace(H + 3.0, 1e6, 97):
            assert F.sigma_of(H, pw) == pytest.approx(O.candidate_sigma(H, pw), rel=1e-9, abs=1e-9), (H, pw)


def test_host_sigma_over_the_whole_range_matches_scipy(F):
    """Significance of any sum, also far below the mean where Q -> 1 (lower tail
    in log1p form), against scipy's regularised incomplete gamma and ndtri."""
    from scipy import special
    for H in (1, 2, 4, 8, 16, 32):
        for S in np.geomspace(0.3, 1e5, 150):
            Q, P = special.gammaincc(H, S), special.gammainc(H, S)
            if min(Q, P) < 1e-290:
                continue
            ref = -special.ndtri(Q) if Q < 0.5 else special.ndtri(P)
            assert F.sigma_of(H, S) == pytest.approx(ref, rel=1e-12, abs=1e-12), (H, S)


def test_geometry_matches_oracle_and_rejects_bad_arguments(F):
    for N, ts, zmax, dz in ((1 << 17, 2e-4, 20.0, 2.0), (1 << 18, 2e-4, 200.0, 2.0),
                            (1 << 23, 2.5e-4, 200.0, 2.0), (4096, 1e-3, 0.0, 1.0)):
        rlo, nr, nz = F.geometry(N, ts, zmax, dz)
        assert rlo == O.rlo_bins(N, ts) and nr == N - 2 * rlo
        assert nz == 2 * O.z_index_max(zmax, dz) + 1
    assert F.geometry(1 << 17, 2e-4, 20.0, 2.0) == (27, 131018, 21)
    bad = [(1001, 1e-3, 10.0, 2.0),     # odd
           (4096, 1e-3, 11.0, 2.0),     # zmax not a multiple of dz
           (4096, 0.0, 10.0, 2.0),      # tsamp
           (4096, 1e-3, 10.0, 0.0),     # dz
           (4096, 1.0, 10.0, 2.0)]      # band empty: rlo >= N/2
    for args in bad:
        with pytest.raises(F.FdasError) as e:
            F.geometry(*args)
        assert e.value.status == F.FDAS_E_INVAL


def test_status_strings_and_null_plan(F):
    lib = F.load()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.fdas_status_string(s)
    assert lib.fdas_last_error(None) == b""
    lib.fdas_plan_destroy(None)


def test_plan_create_rejects_bad_arguments_before_touching_a_device(F):
    lib = F.load()
    h = ctypes.c_void_p()
    o = F.default_opts()
    cases = [(1 << 12, 1, 10.0, 2.0, 3), (1 << 12, 0, 10.0, 2.0, 1), (1 << 12, 1, 11.0, 2.0, 1),
             (1001, 1, 10.0, 2.0, 1)]
    for args in cases:
        assert lib.fdas_plan_create(ctypes.byref(h), *args, ctypes.byref(o)) == F.FDAS_E_INVAL
        assert not h.value
    o.reserved[0] = 1
    assert lib.fdas_plan_create(ctypes.byref(h), 1 << 12, 1, 10.0, 2.0, 1, ctypes.byref(o)) == F.FDAS_E_INVAL
    o = F.default_opts(fail_alloc=-1)
    assert lib.fdas_plan_create(ctypes.byref(h), 1 << 12, 1, 10.0, 2.0, 1, ctypes.byref(o)) == F.FDAS_E_INVAL
    # a drift range whose templates outgrow the largest correlation segment
    assert lib.fdas_plan_create(ctypes.byref(h), 1 << 12, 1, 8000.0, 2.0, 1, None) == F.FDAS_E_UNSUPPORTED
    assert not h.value


def test_plan_create_past_the_argument_checks_without_a_device(F):
    """Valid arguments on a machine without a GPU: the half-built plan is released
    and the call reports a device error (run under the sanitizers by
    test_sanitize_cpu, which would flag a use after free or double free)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = F.load()
    h = ctypes.c_void_p()
    for _ in range(3):
        assert lib.fdas_plan_create(ctypes.byref(h), 1 << 12, 2, 10.0, 2.0, 4, None) == F.FDAS_E_DEVICE
        assert not h.value
