"""Refinement kernels (objective, gradients, ascent) against the FP64 oracle.

Tolerances: P within 1e-4 max(P, 1) (the plane rule); gradients within
1e-3 (|g_ref| + s P) with s_r = 1, s_z = 0.1 (the floor is needed because the
gradient vanishes at a peak); refined points either agree with the oracle's to
2e-3 bins in r and 2e-2 in z, or are at least as good by the oracle's own
objective (both sides may stop at different points of a flat ridge).
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _spec_tensor(Ah):
    import torch
    return torch.from_numpy(np.ascontiguousarray(Ah.astype(np.complex64))).cuda()[None, :]


def _cuda(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _points(Ah, n, seed, zlim=30.0, dz=2.0):
    rng = np.random.default_rng(seed)
    nb = Ah.shape[0] - 1
    pts = []
    for _ in range(n):
        z0 = float(rng.uniform(-zlim, zlim))
        k0 = int(rng.integers(2, nb - 2))
        r = k0 + float(rng.uniform(-1.4, 1.4))
        z = z0 + float(rng.uniform(-2 * dz, 2 * dz))
        pts.append((k0, O.refine_window(z0, dz), r, z))
    # edge cases: zero and tiny drift, windows over bin 0 and past N/2, integer r
    pts += [(40, 19, 40.0, 0.0), (41, 19, 41.3, 1e-5), (9, 20, 9.4, -3e-4), (3, 25, 3.2, 7.0),
            (nb - 2, 22, nb - 2.3, -9.0), (nb - 1, 19, nb - 0.6, 0.5), (500, 18, 500.5, 0.0),
            (777, 30, 777.0, -24.0)]
    return pts


def _eval_gpu(F, spec, pts):
    import torch
    k0 = np.array([p[0] for p in pts], np.int64)
    m = np.array([p[1] for p in pts], np.int32)
    r = np.array([p[2] for p in pts])
    z = np.array([p[3] for p in pts])
    ser = np.zeros(len(pts), np.int32)
    P = F.refine_power(spec, _cuda(r, torch.float64), _cuda(z, torch.float64), _cuda(ser, torch.int32),
                       _cuda(k0, torch.int64), _cuda(m, torch.int32))
    return P.cpu().numpy()


def _check_grad(g, gref, P, s):
    assert abs(g - gref) <= 1e-3 * (abs(gref) + s * P), (g, gref, P)


def test_objective_and_gradients_match_oracle(fdas_gpu):
    import torch
    F = fdas_gpu
    wl = synth.small_batch(1, 1 << 14, 1e-3, 30.0, 2.0, 1, config=99, signals=1, amp_range=(0.5, 0.8))
    Ah = O.normalise(O.spectrum(synth.generate(wl)[0]))[0]
    spec = _spec_tensor(Ah).requires_grad_(False)
    pts = _points(Ah, 120, 1)
    n = len(pts)
    r = _cuda(np.array([p[2] for p in pts]), torch.float64).requires_grad_(True)
    z = _cuda(np.array([p[3] for p in pts]), torch.float64).requires_grad_(True)
    k0 = _cuda(np.array([p[0] for p in pts]), torch.int64)
    m = _cuda(np.array([p[1] for p in pts]), torch.int32)
    ser = torch.zeros(n, dtype=torch.int32, device="cuda")
    P = F.refine_power(spec, r, z, ser, k0, m)
    P.sum().backward()
    Pg = P.detach().cpu().numpy()
    gr = r.grad.cpu().numpy()
    gz = z.grad.cpu().numpy()
    for i, (kk, mm, rr, zz) in enumerate(pts):
        Pr, dr, dzz, _ = O.refine_power(Ah, rr, zz, kk, mm)
        assert abs(Pg[i] - Pr) <= 1e-4 * max(Pr, 1.0), (i, pts[i], Pg[i], Pr)
        _check_grad(gr[i], dr, Pr, 1.0)
        _check_grad(gz[i], dzz, Pr, 0.1)


def test_gradients_match_finite_differences(fdas_gpu):
    """GPU analytic gradients against FP64 central differences (h = 1e-3) of the objective."""
    import torch
    F = fdas_gpu
    rng = np.random.default_rng(5)
    Ah = O.normalise(O.spectrum(rng.standard_normal(1 << 13)))[0]
    spec = _spec_tensor(Ah)
    pts = _points(Ah, 24, 6, zlim=12.0)
    r = _cuda(np.array([p[2] for p in pts]), torch.float64).requires_grad_(True)
    z = _cuda(np.array([p[3] for p in pts]), torch.float64).requires_grad_(True)
    k0 = _cuda(np.array([p[0] for p in pts]), torch.int64)
    m = _cuda(np.array([p[1] for p in pts]), torch.int32)
    ser = torch.zeros(len(pts), dtype=torch.int32, device="cuda")
    F.refine_power(spec, r, z, ser, k0, m).sum().backward()
    h = 1e-3
    for i, (kk, mm, rr, zz) in enumerate(pts):
        P = O.refine_power(Ah, rr, zz, kk, mm)[0]
        fr = (O.refine_power(Ah, rr + h, zz, kk, mm)[0] - O.refine_power(Ah, rr - h, zz, kk, mm)[0]) / (2 * h)
        fz = (O.refine_power(Ah, rr, zz + h, kk, mm)[0] - O.refine_power(Ah, rr, zz - h, kk, mm)[0]) / (2 * h)
        _check_grad(float(r.grad[i]), fr, P, 1.0)
        _check_grad(float(z.grad[i]), fz, P, 0.1)


def test_spectrum_gradient_matches_oracle(fdas_gpu):
    """Weighted sum of P over points sharing bins: d/dA accumulated by the backward kernel."""
    import torch
    F = fdas_gpu
    rng = np.random.default_rng(8)
    Ah = O.normalise(O.spectrum(rng.standard_normal(1 << 12)))[0]
    spec = _spec_tensor(Ah).requires_grad_(True)
    pts = [(300, 20, 300.2, 3.0), (302, 20, 301.7, -5.0), (305, 24, 305.4, 10.0), (900, 18, 900.0, 0.0),
           (3, 22, 2.6, 4.0), (2046, 19, 2046.4, -1.0)]
    w = np.array([1.0, -0.5, 2.0, 0.7, 1.3, -1.1])
    r = _cuda(np.array([p[2] for p in pts]), torch.float64)
    z = _cuda(np.array([p[3] for p in pts]), torch.float64)
    k0 = _cuda(np.array([p[0] for p in pts]), torch.int64)
    m = _cuda(np.array([p[1] for p in pts]), torch.int32)
    ser = torch.zeros(len(pts), dtype=torch.int32, device="cuda")
    P = F.refine_power(spec, r, z, ser, k0, m)
    (P * _cuda(w, torch.float32)).sum().backward()
    got = spec.grad[0].cpu().numpy().astype(np.complex128)
    ref = np.zeros(Ah.shape, np.complex128)
    Pmax = 0.0
    for wi, (kk, mm, rr, zz) in zip(w, pts):
        ks, g = O.refine_spec_grad(Ah, rr, zz, kk, mm)
        ok = (ks >= 0) & (ks < Ah.shape[0])
        np.add.at(ref, ks[ok], wi * g[ok])
        Pmax = max(Pmax, O.refine_power(Ah, rr, zz, kk, mm)[0])
    scale = np.sqrt(Pmax) * 2 * np.abs(w).sum()
    assert np.max(np.abs(got - ref)) <= 1e-4 * scale
    assert got[0] == 0 and got[-1] == 0


def test_large_r_uses_exact_phase(fdas_gpu):
    """Spectrum of a 2^23-sample series (bins to 4.2e6): phases must stay exact at large r."""
    import torch
    F = fdas_gpu
    rng = np.random.default_rng(9)
    nb = 1 << 22
    Ah = np.zeros(nb + 1, np.complex128)
    Ah[1:nb] = (rng.standard_normal(nb - 1) + 1j * rng.standard_normal(nb - 1)) / math.sqrt(2)
    spec = _spec_tensor(Ah)
    pts = [(4100000, 21, 4100000.37, 5.5), (4194300, 19, 4194299.8, 1.0), (3999999, 40, 4000000.2, -42.0),
           (2500000, 18, 2500000.5, 0.0)]
    Pg = _eval_gpu(F, spec, pts)
    for i, (kk, mm, rr, zz) in enumerate(pts):
        Pr = O.refine_power(Ah, rr, zz, kk, mm)[0]
        assert abs(Pg[i] - Pr) <= 1e-4 * max(Pr, 1.0), (pts[i], Pg[i], Pr)


def test_out_of_range_points_give_nan(fdas_gpu):
    import torch
    F = fdas_gpu
    Ah = O.normalise(O.spectrum(np.random.default_rng(1).standard_normal(1 << 12)))[0]
    spec = _spec_tensor(Ah)
    pts = [(100, 20, 100.2, 1.0), (100, 40, 100.2, 1.0), (100, 20, 300.0, 1.0), (100, 20, 100.0, 9000.0)]
    r = _cuda(np.array([p[2] for p in pts]), torch.float64)
    z = _cuda(np.array([p[3] for p in pts]), torch.float64)
    k0 = _cuda(np.array([p[0] for p in pts]), torch.int64)
    m = _cuda(np.array([p[1] for p in pts]), torch.int32)
    ser = torch.zeros(4, dtype=torch.int32, device="cuda")
    P = F.refine_power(spec, r, z, ser, k0, m, max_m=30).cpu().numpy()
    assert np.isfinite(P[0]) and np.all(np.isnan(P[1:]))
    ser[0] = 3                                                  # series out of range
    assert np.isnan(F.refine_power(spec, r[:1], z[:1], ser[:1], k0[:1], m[:1]).cpu().numpy()[0])


def _c1(noise):
    wl = synth.config1(noise=noise)
    x = synth.generate(wl)
    Ah = O.normalise(O.spectrum(x[0]), "median" if noise else "fixed", 1.0)[0]
    rlo = O.rlo_bins(wl.nsamp, wl.tsamp)
    pl = O.plane(Ah, rlo, wl.zmax, wl.dz, method="fft")
    starts = O.refine_starts(pl, rlo, O.z_index_max(wl.zmax, wl.dz), 4096)
    return wl, x, Ah, starts


def test_noise_free_injection_refines_to_truth(fdas_gpu):
    wl, x, _, starts = _c1(False)
    inj = wl.injections[0]
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1, norm="fixed", fixed_var=1.0)
    R, Zq = starts[0]
    r, z, P = plan.refine(_cuda(x, __import__("torch").float32), [R / 2], [Zq * wl.dz])
    assert abs(r[0] - inj.r0) <= 0.01 and abs(z[0] - inj.z0) <= 0.05, (r, z, P)


def test_refinement_matches_oracle_on_single_series_workload(fdas_gpu):
    import torch
    wl, x, Ah, starts = _c1(True)
    inj = wl.injections[0]
    plan = fdas_gpu.Plan(wl.nsamp, 1, wl.zmax, wl.dz, 1)
    r0 = np.array([s[0] / 2 for s in starts])
    z0 = np.array([s[1] * wl.dz for s in starts])
    r, z, P = plan.refine(_cuda(x, torch.float32), r0, z0)
    assert np.all(np.abs(r - r0) <= 1 + 1e-9) and np.all(np.abs(z - z0) <= 2 * wl.dz + 1e-9)
    near = np.nonzero((np.abs(r0 - inj.r0) <= 1) & (np.abs(z0 - inj.z0) <= 2 * wl.dz))[0]
    assert near.size
    i = near[0]
    assert abs(r[i] - inj.r0) <= 0.1 and abs(z[i] - inj.z0) <= 1.0, (r[i], z[i])
    rng = np.random.default_rng(10)
    check = sorted(set(rng.choice(len(starts), 40, replace=False).tolist()) | {0, 1, 2, int(i)})
    for j in check:
        ro, zo, Po = O.refine(Ah, r0[j], z0[j], wl.dz)
        k0, M = int(math.floor(r0[j] + 0.5)), O.refine_window(z0[j], wl.dz)
        Pg_by_oracle = O.refine_power(Ah, r[j], z[j], k0, M)[0]
        assert abs(P[j] - Pg_by_oracle) <= 1e-4 * max(Pg_by_oracle, 1.0)
        same = abs(r[j] - ro) <= 2e-3 and abs(z[j] - zo) <= 2e-2
        assert same or Pg_by_oracle >= Po * (1 - 1e-4), (j, (r[j], z[j], P[j]), (ro, zo, Po))


def test_refine_rejects_bad_starts(fdas_gpu):
    import torch
    F = fdas_gpu
    x = _cuda(np.random.default_rng(2).standard_normal((2, 1 << 12)), torch.float32)
    plan = F.Plan(1 << 12, 2, 10.0, 2.0, 1)
    for kw in (dict(series=[5]), dict(r0=[-3.0]), dict(r0=[5000.0]), dict(z0=[9000.0]), dict(z0=[float("nan")])):
        args = dict(r0=[100.0], z0=[2.0], series=[0])
        args.update(kw)
        with pytest.raises(F.FdasError) as e:
            plan.refine(x, args["r0"], args["z0"], series=args["series"])
        assert e.value.status == F.FDAS_E_INVAL
    r, z, P = plan.refine(x, np.zeros(0), np.zeros(0))
    assert r.size == 0
