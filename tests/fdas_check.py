"""Comparison rules between the HIP path and the FP64 oracle.

Plane powers: |P_gpu - P_ora| <= 1e-4 * max(P_ora, 1) (the floor is the mean
noise power: a relative error of a power near zero is meaningless, and FP32
FFT round-off is absolute at the level of the segment's total power).

Candidates: one per (series, harm, r_idx). Key sets must be identical except
for columns whose oracle maximum lies within a relative 1e-4 of the stage
threshold (either side may then legitimately decide differently). For common
keys the powers agree within 1e-4, and the reported drift index is either the
oracle's or one whose oracle sum is within 1e-4 of the column maximum (ties
between drift rows).
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np

import oracle as O

REL = 1e-4


class OracleSeries:
    """Full oracle results of one series: plane and per-stage column maxima."""

    def __init__(self, x, tsamp, zmax, dz, numharm, norm="median", fixed_var=1.0, K=16,
                 method=None, plane=None):
        x = np.asarray(x)
        self.N = x.shape[-1]
        self.tsamp, self.zmax, self.dz, self.numharm = tsamp, zmax, dz, numharm
        self.rlo = O.rlo_bins(self.N, tsamp)
        self.Z = O.z_index_max(zmax, dz)
        if method is None:
            method = "direct" if self.N <= (1 << 15) else "fft"
        if plane is None and norm == "local":
            self.Ah, _ = O.deredden(O.spectrum(x))
            self.norm = float("nan")
            self.plane = O.plane(self.Ah, self.rlo, zmax, dz, K, method)
        elif plane is None:
            self.Ah, self.norm = O.normalise(O.spectrum(x), norm, fixed_var)
            self.plane = O.plane(self.Ah, self.rlo, zmax, dz, K, method)
        else:
            self.plane = np.asarray(plane, dtype=np.float64)
        self.stages: Dict[int, tuple] = {}
        for H in O.stage_list(numharm):
            self.stages[H] = O.stage_maxima(self.plane, self.rlo, self.Z, H, self.N)

    def column(self, H, R):
        Rs, M, Zs = self.stages[H]
        i = R - Rs[0]
        return M[i], Zs[i]

    def sum_at(self, H, R, Zq):
        S = O.stage_sums_at(self.plane, self.rlo, self.Z, H, [R])
        return S[Zq + self.Z, 0]

    def candidates(self, sigma):
        out = []
        for H, (Rs, M, Zs) in self.stages.items():
            T = O.threshold(H, sigma)
            for i in np.nonzero(M > T)[0]:
                out.append((H, int(Rs[i]), int(Zs[i]), float(M[i])))
        return out


def assert_plane_close(gpu, ora, rel=REL):
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    assert gpu.shape == ora.shape, (gpu.shape, ora.shape)
    err = np.abs(gpu - ora) / np.maximum(ora, 1.0)
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= rel, f"max rel err {err.max():.3e} at {worst}: gpu {gpu[worst]} ora {ora[worst]}"
    return float(err.max())


def assert_candidates_match(gpu_cands, oracles: Dict[int, OracleSeries], sigma, rel=REL):
    """gpu_cands: structured array from the binding; oracles: series index -> OracleSeries."""
    g = {}
    for c in gpu_cands:
        key = (int(c["series"]), int(c["harm"]), int(c["r_idx"]))
        assert key not in g, f"duplicate candidate {key}"
        g[key] = (int(c["z_idx"]), float(c["power"]))
    o = {}
    for b, orc in oracles.items():
        for H, R, Zq, M in orc.candidates(sigma):
            o[(b, H, R)] = (Zq, M)
    gpu_series = {k[0] for k in g}
    assert gpu_series <= set(oracles), f"candidates for unchecked series {gpu_series - set(oracles)}"
    banded = 0
    for key in set(g) ^ set(o):
        b, H, R = key
        M, _ = oracles[b].column(H, R)
        T = O.threshold(H, sigma)
        if abs(M - T) <= rel * T:
            banded += 1
            continue
        side = "gpu only" if key in g else "oracle only"
        raise AssertionError(f"{side} candidate {key}: oracle M={M:.6f} T={T:.6f} gpu={g.get(key)}")
    for key in set(g) & set(o):
        b, H, R = key
        zg, pg = g[key]
        zo, po = o[key]
        assert abs(pg - po) <= rel * max(po, 1.0), f"{key}: power gpu {pg} oracle {po}"
        if zg != zo:
            s = oracles[b].sum_at(H, R, zg)
            assert s >= po * (1 - rel), f"{key}: z gpu {zg} (oracle sum {s}) vs oracle {zo} ({po})"
    # sorted by (series, harm, r_idx)
    keys = [(int(c["series"]), int(c["harm"]), int(c["r_idx"])) for c in gpu_cands]
    assert keys == sorted(keys)
    return len(set(g) & set(o)), banded
