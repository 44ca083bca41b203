"""Plain references of the post-search steps: red-noise normalisation and sifting.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 2 of the paper sifts the accelsearch results (ACCEL_sift) before
folding; the paper states neither step's rules. The readings adopted here:

Local-median normalisation ("dereddening"), an alternative to the global
median for spectra with red noise:
  * bins 1..N/2-1 are cut into consecutive blocks starting at b_0 = 1, block i
    of width w_i = min(200, 6 + floor(b_i / 30)) (the last block ends at N/2);
  * m_i = (lower median of |A_k|^2 over block i) / ln 2, placed at the block
    centre c_i = (b_i + e_i - 1)/2 (e_i the block end, exclusive);
  * m(k) interpolates m_i linearly between neighbouring centres and is constant
    below the first and above the last centre;
  * A^_k = A_k / sqrt(m(k)) (zero where m(k) = 0), A^_0 = A^_{N/2} = 0.

Sifting of a candidate list (any mix of series, e.g. the trial DMs of one
observation), on the fundamental frequency f (Hz) and significance sigma:
  * order: sigma descending, then series, harm, r_idx ascending;
  * duplicates: walking that order, a candidate within tol / min(T_a, T_b) Hz of
    an already kept candidate joins the first such kept candidate (which counts
    it); otherwise it is kept (tol in Fourier bins, T the observation length);
  * harmonics: walking the kept candidates in the same order, B is dropped when
    a stronger kept, not dropped A has |f_B - rho f_A| <= rho tol / min(T_A, T_B)
    for a ratio rho = n or 1/n, 2 <= n <= max_ratio (integer harmonics and
    subharmonics only: ratios p/q with both p, q > 1 are so dense that almost
    any frequency would lie near one of them);
  * the result lists the surviving candidates in that order with their hit
    counts (themselves plus the duplicates they absorbed) and the smallest and
    largest series index among them.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

__all__ = ["deredden_blocks", "deredden", "sift"]

LN2 = math.log(2.0)


def deredden_blocks(half: int) -> List[Tuple[int, int]]:
    """Blocks [b, e) covering bins 1..half-1: width min(200, 6 + b // 30)."""
    out = []
    b = 1
    while b < half:
        w = min(200, 6 + b // 30)
        e = min(half, b + w)
        out.append((b, e))
        b = e
    return out


def deredden(A: np.ndarray):
    """(A^, m): locally normalised spectrum and the per-bin mean-power estimate m(k)."""
    A = np.asarray(A, dtype=np.complex128)
    half = A.shape[-1] - 1
    pw = A.real ** 2 + A.imag ** 2
    blocks = deredden_blocks(half)
    cen = np.array([(b + e - 1) / 2.0 for b, e in blocks])
    med = np.empty(len(blocks))
    for i, (b, e) in enumerate(blocks):
        s = np.sort(pw[b:e])
        med[i] = s[(e - b - 1) // 2] / LN2
    m = np.empty(half + 1)
    for kk in range(1, half):
        if kk <= cen[0]:
            m[kk] = med[0]
        elif kk >= cen[-1]:
            m[kk] = med[-1]
        else:
            i = int(np.searchsorted(cen, kk, side="right")) - 1      # cen[i] <= kk < cen[i+1]
            f = (kk - cen[i]) / (cen[i + 1] - cen[i])
            m[kk] = med[i] + (med[i + 1] - med[i]) * f
    m[0] = m[half] = 0.0
    Ah = np.zeros_like(A)
    ok = m > 0
    ok[0] = ok[half] = False
    Ah[ok] = A[ok] / np.sqrt(m[ok])
    return Ah, m


def _order(cands) -> List[int]:
    return sorted(range(len(cands)), key=lambda i: (-float(cands[i]["sigma"]), int(cands[i]["series"]),
                                                   int(cands[i]["harm"]), int(cands[i]["r_idx"])))


def _tobs(c) -> float:
    return float(c["r_fund"]) / float(c["f_hz"])


def sift(cands, tol_bins: float = 1.1, max_ratio: int = 16):
    """Sifted list: [(index into cands, hits, min series, max series)] in sifted order."""
    order = _order(cands)
    kept: List[int] = []
    hits: Dict[int, int] = {}
    lo: Dict[int, int] = {}
    hi: Dict[int, int] = {}
    for i in order:
        f, T = float(cands[i]["f_hz"]), _tobs(cands[i])
        home = None
        for j in kept:                                  # kept in order: the first match wins
            if abs(f - float(cands[j]["f_hz"])) <= tol_bins / min(T, _tobs(cands[j])):
                home = j
                break
        s = int(cands[i]["series"])
        if home is None:
            kept.append(i)
            hits[i], lo[i], hi[i] = 1, s, s
        else:
            hits[home] += 1
            lo[home] = min(lo[home], s)
            hi[home] = max(hi[home], s)
    ratios = [(n, 1) for n in range(2, max_ratio + 1)] + [(1, n) for n in range(2, max_ratio + 1)]
    alive: List[int] = []
    for b in kept:
        fb, Tb = float(cands[b]["f_hz"]), _tobs(cands[b])
        harmonic = False
        for a in alive:                                 # stronger survivors only
            fa, Ta = float(cands[a]["f_hz"]), _tobs(cands[a])
            tol = tol_bins / min(Ta, Tb)
            for p, q in ratios:
                if abs(fb - p / q * fa) <= p / q * tol:
                    harmonic = True
                    break
            if harmonic:
                break
        if not harmonic:
            alive.append(b)
    return [(i, hits[i], lo[i], hi[i]) for i in alive]
