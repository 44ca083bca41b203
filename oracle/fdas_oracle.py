"""Plain FP64 reference of the acceleration-search hot path.

TEST INFRASTRUCTURE ONLY (see the package docstring). Slow on purpose: each
function is the plain definition of one step, written so that it can be
checked against the definitions by eye. Library primitives used as steps:
numpy's FFT (checked against the direct DFT), scipy's Fresnel integrals
(checked against quadrature of the defining integral), scipy's FFT
convolution (checked against the direct tap sum) and a sort (the median).

Paper context: Section 2 lists the pipeline; step 3 takes the FFT of each
dedispersed series (realfft), step 4 searches it for periodic signals with a
frequency derivative bounded by zmax (accelsearch; zmax is the knob of
Section 3.2 / Table 4), step 5 collects candidates. The paper does not state
the mathematics of steps 3-5; the conventions below are the readings adopted
for them:

  * spectrum     A_k = sum_n x_n exp(-2 pi i k n / N), k = 0..N/2;
  * normalise    norm = (lower median of |A_k|^2, k = 1..N/2-1) / ln 2,
                 A^_k = A_k / sqrt(norm), A^_0 = A^_{N/2} = 0, zero outside;
  * response     rho(q, z) = int_0^1 exp(2 pi i [q u + z (u^2 - u)/2]) du,
                 r is the Fourier frequency at mid-observation, z the total
                 drift in bins over the observation;
  * power        P(r, z) = |sum_k A^_k t_k|^2 / E with t_k = conj rho(r-k, z)
                 over |k - r| <= m(z) = ceil(|z|/2) + K and E = sum |t_k|^2;
  * grid         r = R/2 (half bins), R in [2 rlo, N-1], rlo = ceil(flo T);
                 z = Zq dz, Zq in [-zmax/dz, zmax/dz];
  * harmonics    S_H(R, Zq) = sum_{k=1..H} P(R_k, Zq_k),
                 R_k = floor((2 R k + H) / (2 H)),
                 Zq_k = sgn(Zq) floor((2 |Zq| k + H) / (2 H)),
                 H in {1, 2, 4, ..., numharm}, R in [2 rlo H, N-1];
  * maxima       M_H(R) = max_Zq S_H(R, Zq), Zq* the smallest maximiser;
  * threshold    candidate iff M_H(R) > T_H, where Q(H, T_H) = p,
                 Q(H, S) = exp(-S) sum_{j<H} S^j / j! (survival of a sum of H
                 unit exponentials) and p = erfc(sigma / sqrt 2) / 2.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np
from scipy import signal as _sig
from scipy import special as _sp

__all__ = [
    "rlo_bins", "z_index_max", "half_width", "rho", "rho_quad", "dft_direct", "spectrum",
    "normalise", "template", "plane", "plane_cells", "harmonic_index", "stage_list",
    "stage_maxima", "stage_sums_at", "gamma_sf", "log_gamma_sf", "threshold",
    "candidate_sigma", "search", "search_series", "CAND_FIELDS", "window_maxima",
    "plane_band", "band_maxima",
]

LN2 = math.log(2.0)


# ----------------------------------------------------------------------------- grid

def rlo_bins(nsamp: int, tsamp: float, flo: float = 1.0) -> int:
    """Lowest searched Fourier bin: ceil(flo * T), T = nsamp * tsamp, at least 1."""
    T = float(nsamp) * float(tsamp)
    return max(1, int(math.ceil(float(flo) * T)))


def z_index_max(zmax: float, dz: float) -> int:
    """Zmax = zmax/dz, which must be a whole number; the z grid is Zq*dz, |Zq| <= Zmax."""
    q = float(zmax) / float(dz)
    Z = int(round(q))
    if dz <= 0 or zmax < 0 or abs(q - Z) > 1e-9 * max(1.0, abs(q)):
        raise ValueError("zmax must be a non-negative whole multiple of dz > 0")
    return Z


def half_width(z: float, K: int = 16) -> int:
    """Template half-width in bins: m(z) = ceil(|z|/2) + K."""
    return int(math.ceil(abs(float(z)) / 2.0)) + int(K)


# ----------------------------------------------------------------------------- response

def rho_quad(q, z: float, order: int = 16) -> np.ndarray:
    """rho(q, z) by composite Gauss-Legendre quadrature of its defining integral.

    rho(q, z) = int_0^1 exp(2 pi i [q u + z (u^2 - u)/2]) du. Panels are sized so
    that the phase turns by at most ~1 rad per panel.
    """
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    z = float(z)
    xg, wg = np.polynomial.legendre.leggauss(order)
    out = np.empty(q.shape, dtype=np.complex128)
    for i, qq in enumerate(q.ravel()):
        npan = int(math.ceil(math.pi * (abs(qq) + abs(z) / 2.0 + 1.0))) + 4
        edges = np.linspace(0.0, 1.0, npan + 1)
        a = edges[:-1][:, None]
        h = (edges[1] - edges[0])
        u = a + 0.5 * h * (xg[None, :] + 1.0)
        ph = 2.0 * np.pi * (qq * u + z * (u * u - u) * 0.5)
        out.ravel()[i] = 0.5 * h * np.sum(wg[None, :] * np.exp(1j * ph))
    return out


def rho(q, z: float) -> np.ndarray:
    """Response of a drifting sinusoid at offset q = r0 - k bins and drift z.

    Closed form (complete the square in the defining integral): for z > 0,
    rho = exp(-i pi (q - z/2)^2 / z) / sqrt(2 z) *
          [(C(Ye) - C(Ys)) + i (S(Ye) - S(Ys))],  Y(e,s) = (q +- z/2) sqrt(2/z),
    with C, S the Fresnel integrals of argument pi t^2 / 2. For z < 0 the
    defining integral gives rho(q, z) = conj rho(-q, -z); at z = 0 it is
    exp(i pi q) sinc(q). Below |z| = 1e-3 the closed form cancels badly and the
    quadrature of the definition is used instead.
    """
    q = np.asarray(q, dtype=np.float64)
    z = float(z)
    if z == 0.0:
        return np.exp(1j * np.pi * q) * np.sinc(q)
    if z < 0.0:
        return np.conj(rho(-q, -z))
    if z < 1e-3:
        return rho_quad(q, z).reshape(q.shape)
    s = math.sqrt(2.0 / z)
    ye = (q + z / 2.0) * s
    ys = (q - z / 2.0) * s
    se, ce = _sp.fresnel(ye)
    ss, cs = _sp.fresnel(ys)
    pref = np.exp(-1j * np.pi * (q - z / 2.0) ** 2 / z) / math.sqrt(2.0 * z)
    return pref * ((ce - cs) + 1j * (se - ss))


# ----------------------------------------------------------------------------- spectrum

def dft_direct(x) -> np.ndarray:
    """A_k = sum_n x_n exp(-2 pi i k n / N), k = 0..N/2, by the direct sum (small N only)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    k = np.arange(N // 2 + 1)[:, None]
    n = np.arange(N)[None, :]
    ang = 2.0 * np.pi * ((k * n) % N) / N      # exact integer reduction of k n mod N
    return (x[None, :] * np.exp(-1j * ang)).sum(axis=1)


def spectrum(x) -> np.ndarray:
    """A_k, k = 0..N/2, of a real series in FP64 (numpy's real FFT, same sign as above)."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[-1] % 2:
        raise ValueError("nsamp must be even")
    return np.fft.rfft(x)


def normalise(A: np.ndarray, mode: str = "median", fixed_var: float = 1.0):
    """Return (A^, norm): A^_k = A_k / sqrt(norm) for k in [1, N/2-1], 0 at DC and Nyquist.

    median: norm = s_(floor((M-1)/2)) / ln 2 with s the ascending |A_k|^2 over the
            M = N/2 - 1 bins k = 1..N/2-1 (the lower median; the median of a
            unit exponential is ln 2, so white noise maps to unit mean power);
    fixed : norm = N * fixed_var (the exact mean of |A_k|^2 for white noise).
    A median of zero (e.g. an all-zero series) leaves all powers at zero.
    """
    A = np.asarray(A, dtype=np.complex128)
    half = A.shape[-1] - 1            # N/2
    N = 2 * half
    if mode == "median":
        pw = np.sort(A[1:half].real ** 2 + A[1:half].imag ** 2)
        M = pw.shape[0]
        norm = float(pw[(M - 1) // 2]) / LN2
    elif mode == "fixed":
        norm = float(N) * float(fixed_var)
    else:
        raise ValueError(mode)
    if norm <= 0.0:
        # a series whose median power is zero carries no searchable power
        return np.zeros_like(A), norm
    Ah = A / math.sqrt(norm)
    Ah[0] = 0.0
    Ah[half] = 0.0
    return Ah, norm


# ----------------------------------------------------------------------------- plane

def template(z: float, parity: int, K: int = 16):
    """Unit-energy taps for a trial at r = k0 + parity/2, drift z.

    Returns (d, t): tap offsets d = k - k0 with |k - r| <= m(z), i.e.
    d in [-m + parity, m], and t_d = conj rho(parity/2 - d, z) / sqrt(E).
    """
    m = half_width(z, K)
    d = np.arange(-m + parity, m + 1)
    t = np.conj(rho(parity / 2.0 - d, z))
    E = float(np.sum(t.real ** 2 + t.imag ** 2))
    return d, t / math.sqrt(E)


def _padded(Ah: np.ndarray, pad: int) -> np.ndarray:
    out = np.zeros(Ah.shape[-1] + 2 * pad, dtype=np.complex128)
    out[pad:pad + Ah.shape[-1]] = Ah
    return out


def plane(Ah: np.ndarray, rlo: int, zmax: float, dz: float, K: int = 16,
          method: str = "direct", dtype=np.float64) -> np.ndarray:
    """Power plane P[zi][R - 2 rlo], zi = Zq + Zmax, R in [2 rlo, N-1].

    direct: c(k0) = sum_d A^_{k0+d} t_d, one shifted vector product per tap;
    fft   : the same correlation through scipy's FP64 FFT convolution.
    """
    half = Ah.shape[-1] - 1
    N = 2 * half
    Z = z_index_max(zmax, dz)
    NR = N - 2 * rlo
    if NR <= 0:
        raise ValueError("no searchable bins")
    k0 = np.arange(rlo, half)                 # integer part of r; r = k0 + p/2
    mmax = half_width(Z * dz, K)
    pad = mmax + 2
    Ap = _padded(Ah, pad)
    out = np.zeros((2 * Z + 1, NR), dtype=dtype)
    for zi in range(2 * Z + 1):
        z = (zi - Z) * dz
        for p in (0, 1):
            d, t = template(z, p, K)
            if method == "direct":
                c = np.zeros(k0.shape[0], dtype=np.complex128)
                for dd, tt in zip(d, t):
                    c += Ap[k0 + dd + pad] * tt
            elif method == "fft":
                # y[n] = sum_j Ap[n - j] t[-1 - j]  =>  c(k0) = y[k0 + pad + d[-1]]
                y = _sig.fftconvolve(Ap, t[::-1], mode="full")
                c = y[k0 + pad + d[-1]]
            else:
                raise ValueError(method)
            out[zi, 2 * (k0 - rlo) + p] = c.real ** 2 + c.imag ** 2
    return out


def plane_cells(Ah: np.ndarray, R: Sequence[int], Zq: Sequence[int], dz: float,
                K: int = 16) -> np.ndarray:
    """P at the listed cells (R half bins, Zq z-steps), each by its own direct tap sum.

    Cells sharing a template (same Zq and parity) are evaluated together; every
    cell is still the plain sum over its own taps.
    """
    R = np.asarray(R, dtype=np.int64)
    Zq = np.asarray(Zq, dtype=np.int64)
    out = np.empty(R.shape[0], dtype=np.float64)
    half = Ah.shape[-1] - 1
    if R.shape[0] == 0:
        return out
    key = Zq * 2 + (R & 1)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    bounds = np.nonzero(np.diff(ks))[0] + 1
    for grp in np.split(order, bounds):
        z = float(Zq[grp[0]]) * dz
        p = int(R[grp[0]] & 1)
        d, t = template(z, p, K)
        k = (R[grp] >> 1)[:, None] + d[None, :]
        ok = (k >= 1) & (k <= half - 1)
        vals = np.where(ok, Ah[np.clip(k, 0, half)], 0.0)
        c = np.sum(vals * t[None, :], axis=1)
        out[grp] = c.real ** 2 + c.imag ** 2
    return out


# ----------------------------------------------------------------------------- harmonics

def stage_list(numharm: int) -> List[int]:
    """Harmonic stages 1, 2, 4, ..., numharm (numharm a power of two up to 32)."""
    if numharm not in (1, 2, 4, 8, 16, 32):
        raise ValueError("numharm must be one of 1, 2, 4, 8, 16, 32")
    out, h = [], 1
    while h <= numharm:
        out.append(h)
        h *= 2
    return out


def harmonic_index(R, Zq, k: int, H: int):
    """(R_k, Zq_k): the k-th of H harmonics of the trial whose H-th harmonic is (R, Zq).

    R_k = floor((2 R k + H) / (2 H)) rounds R k / H half up; Zq_k rounds Zq k / H
    half away from zero. Integer arithmetic only.
    """
    R = np.asarray(R, dtype=np.int64)
    Zq = np.asarray(Zq, dtype=np.int64)
    Rk = (2 * R * k + H) // (2 * H)
    Zk = np.sign(Zq) * ((2 * np.abs(Zq) * k + H) // (2 * H))
    return Rk, Zk


def stage_sums_at(pl: np.ndarray, rlo: int, Z: int, H: int, R) -> np.ndarray:
    """S_H(R, Zq) for the listed R (all Zq), summed in FP64 in the order k = 1..H."""
    R = np.asarray(R, dtype=np.int64)
    Zq = np.arange(-Z, Z + 1, dtype=np.int64)
    S = np.zeros((Zq.shape[0], R.shape[0]), dtype=np.float64)
    for k in range(1, H + 1):
        Rk, _ = harmonic_index(R, 0, k, H)
        _, Zk = harmonic_index(0, Zq, k, H)
        S += pl[(Zk + Z)[:, None], (Rk - 2 * rlo)[None, :]]
    return S


def stage_maxima(pl: np.ndarray, rlo: int, Z: int, H: int, nsamp: int, chunk: int = 8192):
    """(R, M_H(R), Zq*) for R in [2 rlo H, nsamp-1]; Zq* is the smallest maximiser."""
    Rall = np.arange(2 * rlo * H, nsamp, dtype=np.int64)
    M = np.empty(Rall.shape[0], dtype=np.float64)
    Zs = np.empty(Rall.shape[0], dtype=np.int64)
    for s in range(0, Rall.shape[0], chunk):
        R = Rall[s:s + chunk]
        S = stage_sums_at(pl, rlo, Z, H, R)
        a = np.argmax(S, axis=0)            # first (smallest Zq) maximiser
        M[s:s + chunk] = S[a, np.arange(R.shape[0])]
        Zs[s:s + chunk] = a - Z
    return Rall, M, Zs


# ----------------------------------------------------------------------------- statistics

def log_gamma_sf(H: int, S: float) -> float:
    """log Q(H, S), Q(H, S) = exp(-S) sum_{j<H} S^j / j!, evaluated in log space."""
    S = float(S)
    if S <= 0.0:
        return 0.0
    terms = [j * math.log(S) - math.lgamma(j + 1.0) for j in range(H)]
    mx = max(terms)
    return -S + mx + math.log(sum(math.exp(t - mx) for t in terms))


def gamma_sf(H: int, S: float) -> float:
    """Q(H, S): probability that a sum of H unit exponentials exceeds S."""
    return math.exp(log_gamma_sf(H, S))


def threshold(H: int, sigma: float) -> float:
    """T_H with Q(H, T_H) = p, p = erfc(sigma/sqrt 2)/2, by bisection on log Q."""
    logp = math.log(0.5 * math.erfc(float(sigma) / math.sqrt(2.0)))
    lo, hi = 0.0, 1.0
    while log_gamma_sf(H, hi) > logp:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if log_gamma_sf(H, mid) > logp:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    return 0.5 * (lo + hi)


def candidate_sigma(H: int, power: float) -> float:
    """Gaussian-equivalent single-trial significance of M_H = power: -Phi^-1(Q(H, power))."""
    return float(-_sp.ndtri_exp(log_gamma_sf(H, power)))


# ----------------------------------------------------------------------------- search

CAND_FIELDS = ("series", "harm", "r_idx", "z_idx", "power", "sigma",
               "r_fund", "z_fund", "f_hz", "fdot_hz_s")


def search_series(x, tsamp: float, zmax: float, dz: float, numharm: int, sigma: float,
                  flo: float = 1.0, K: int = 16, norm: str = "median", fixed_var: float = 1.0,
                  method: Optional[str] = None, series: int = 0,
                  return_plane: bool = False):
    """All candidates of one series, sorted by (harm, r_idx)."""
    x = np.asarray(x)
    N = x.shape[-1]
    T = N * float(tsamp)
    rlo = rlo_bins(N, tsamp, flo)
    Z = z_index_max(zmax, dz)
    if method is None:
        method = "direct" if N <= (1 << 17) else "fft"
    Ah, _ = normalise(spectrum(x), norm, fixed_var)
    pl = plane(Ah, rlo, zmax, dz, K, method)
    out = []
    for H in stage_list(numharm):
        TH = threshold(H, sigma)
        R, M, Zs = stage_maxima(pl, rlo, Z, H, N)
        for i in np.nonzero(M > TH)[0]:
            rf = R[i] / (2.0 * H)
            zf = Zs[i] * dz / H
            out.append(dict(series=series, harm=H, r_idx=int(R[i]), z_idx=int(Zs[i]),
                            power=float(M[i]), sigma=candidate_sigma(H, M[i]),
                            r_fund=rf, z_fund=zf, f_hz=rf / T, fdot_hz_s=zf / (T * T)))
    if return_plane:
        return out, pl
    return out


def search(batch, tsamp: float, zmax: float, dz: float, numharm: int, sigma: float,
           series_ids: Optional[Sequence[int]] = None, **kw) -> List[dict]:
    """Candidates of a batch [B][N], sorted by (series, harm, r_idx)."""
    batch = np.atleast_2d(np.asarray(batch))
    ids = list(range(batch.shape[0])) if series_ids is None else list(series_ids)
    out = []
    for row, b in enumerate(ids):
        out.extend(search_series(batch[row], tsamp, zmax, dz, numharm, sigma, series=b, **kw))
    out.sort(key=lambda c: (c["series"], c["harm"], c["r_idx"]))
    return out


def window_maxima(Ah: np.ndarray, rlo: int, zmax: float, dz: float, H: int, R_lo: int,
                  R_hi: int, K: int = 16, R_list: Optional[Sequence[int]] = None):
    """M_H(R), Zq* (and all S_H) for R in [R_lo, R_hi) (or the listed R) from directly
    evaluated plane cells only.

    Evaluates just the cells the H-harmonic sums of those columns read, so it
    works at any series length.
    """
    Z = z_index_max(zmax, dz)
    R = np.arange(R_lo, R_hi, dtype=np.int64) if R_list is None else np.asarray(R_list, dtype=np.int64)
    Zq = np.arange(-Z, Z + 1, dtype=np.int64)
    cellsR, cellsZ = [], []
    for k in range(1, H + 1):
        Rk, _ = harmonic_index(R, 0, k, H)
        _, Zk = harmonic_index(0, Zq, k, H)
        cellsR.append(np.repeat(Rk[None, :], Zq.shape[0], axis=0).ravel())
        cellsZ.append(np.repeat(Zk[:, None], R.shape[0], axis=1).ravel())
    cR = np.concatenate(cellsR)
    cZ = np.concatenate(cellsZ)
    uniq, inv = np.unique(np.stack([cR, cZ], axis=1), axis=0, return_inverse=True)
    vals = plane_cells(Ah, uniq[:, 0], uniq[:, 1], dz, K)[inv.ravel()]
    n = Zq.shape[0] * R.shape[0]
    S = np.zeros((Zq.shape[0], R.shape[0]), dtype=np.float64)
    for k in range(H):
        S += vals[k * n:(k + 1) * n].reshape(Zq.shape[0], R.shape[0])
    a = np.argmax(S, axis=0)
    return R, S[a, np.arange(R.shape[0])], a - Z, S


def plane_band(Ah: np.ndarray, R_lo: int, R_hi: int, zmax: float, dz: float, K: int = 16,
               rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """P[zi][R - R_lo] for the columns R in [R_lo, R_hi) (half bins) and the z rows
    zi = Zq + Zmax listed in rows (default: all; rows not listed stay 0).

    The same definition as plane(): c(k0) = sum_d A^_{k0+d} t_d over the taps of
    the trial (r = k0 + parity/2), bins outside [1, N/2 - 1] read as zero, each
    tap sum a direct (non-FFT) correlation, on a column range only, so that it
    works on series of any length.
    """
    half = Ah.shape[-1] - 1
    Z = z_index_max(zmax, dz)
    if R_hi <= R_lo:
        return np.zeros((2 * Z + 1, 0))
    k_lo, k_hi = R_lo >> 1, (R_hi - 1) >> 1              # trial bins k0 (inclusive)
    pad = half_width(Z * dz, K) + 2
    # spectrum bins k_lo - pad .. k_hi + pad, zero outside [1, N/2 - 1]
    kk = np.arange(k_lo - pad, k_hi + pad + 1)
    ok = (kk >= 1) & (kk <= half - 1)
    seg = np.where(ok, Ah[np.clip(kk, 0, half)], 0.0).astype(np.complex128)
    k0 = np.arange(k_lo, k_hi + 1)
    out = np.zeros((2 * Z + 1, R_hi - R_lo), dtype=np.float64)
    for zi in (range(2 * Z + 1) if rows is None else sorted(set(int(r) for r in rows))):
        z = (zi - Z) * dz
        for p in (0, 1):
            d, t = template(z, p, K)
            # c(k0) = sum_j seg[k0 - k_lo + pad + d_j] t_j: a direct correlation
            lo = pad + int(d[0])
            c = np.convolve(seg[lo:lo + k0.shape[0] + t.shape[0] - 1], t[::-1], mode="valid")
            R = 2 * k0 + p
            sel = (R >= R_lo) & (R < R_hi)
            out[zi, R[sel] - R_lo] = c[sel].real ** 2 + c[sel].imag ** 2
    return out


def band_maxima(Ah: np.ndarray, rlo: int, zmax: float, dz: float, H: int, R_lo: int, R_hi: int,
                K: int = 16, return_sums: bool = False):
    """(R, M_H(R), Zq*) for the contiguous columns R in [R_lo, R_hi) of stage H
    (and S_H[Zq + Zmax][R - R_lo] with return_sums).

    S_H(R, Zq) = sum_{k=1..H} P(R_k, Zq_k) in the order k = 1..H, the plane cells
    of harmonic k taken from plane_band over the columns [R_k(R_lo), R_k(R_hi - 1)]
    and only the rows Zq_k that harmonic reads; Zq* is the smallest maximiser.
    """
    Z = z_index_max(zmax, dz)
    R = np.arange(R_lo, R_hi, dtype=np.int64)
    Zq = np.arange(-Z, Z + 1, dtype=np.int64)
    S = np.zeros((Zq.shape[0], R.shape[0]), dtype=np.float64)
    for k in range(1, H + 1):
        Rk, _ = harmonic_index(R, 0, k, H)
        _, Zk = harmonic_index(0, Zq, k, H)
        lo, hi = int(Rk[0]), int(Rk[-1]) + 1
        pb = plane_band(Ah, lo, hi, zmax, dz, K, rows=Zk + Z)
        S += pb[(Zk + Z)[:, None], (Rk - lo)[None, :]]
    a = np.argmax(S, axis=0)
    if return_sums:
        return R, S[a, np.arange(R.shape[0])], a - Z, S
    return R, S[a, np.arange(R.shape[0])], a - Z
