"""Plain FP64 reference of candidate refinement (power at fractional r and z).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The search of Section 2 (steps 4-5) reports candidates on the half-bin, dz
grid; refining a candidate means maximising the correlation power over
continuous (r, z) near it. The paper does not define this step; the reading
adopted here:

  * objective   P(r, z) = |c(r, z)|^2,  c(r, z) = sum_{k=k0-M}^{k0+M} A^_k conj rho(r - k, z),
                with the window (k0, M) fixed at the start point (r0, z0):
                k0 = nearest bin to r0, M = ceil((|z0| + 2 dz)/2) + K + 1, and no
                renormalisation, so that P is smooth in (r, z) (the plane's
                unit-energy normalisation jumps where its tap set changes);
  * derivatives dc/dr = sum A^_k conj d(rho)/dq (r - k, z), dc/dz likewise with
                d(rho)/dz; dP/dx = 2 Re(conj(c) dc/dx);
  * ascent      (r, z) += (eta_r dP/dr, eta_z dP/dz) / P with eta_r = 3/(2 pi^2),
                eta_z = 90/pi^2 (the Newton steps of ln P at a peak of |rho|^2,
                whose curvatures in q and z are -2 pi^2/3 and -pi^2/90), each
                step clamped to |r - r0| <= 1, |z - z0| <= 2 dz, 20 iterations.

Derivatives of rho(q, z) = int_0^1 exp(2 pi i theta(u)) du, theta = q u + z (u^2 - u)/2:
  d(rho)/dq = 2 pi i I1,  d(rho)/dz = pi i (I2 - I1),  I_n = int_0^1 u^n exp(2 pi i theta) du.
Integrating d/du exp(2 pi i theta) and d/du [u exp(2 pi i theta)] over [0, 1]
(theta' = (q - z/2) + z u, theta(1) = q) gives, for z != 0,
  z I1 = (e^{2 pi i q} - 1)/(2 pi i) - (q - z/2) rho,
  z I2 = (e^{2 pi i q} - rho)/(2 pi i) - (q - z/2) I1.
These divide by z and lose about (q/z)^2 ulps to cancellation; for
|z| < max(1, |q|/16) the integrals are taken by composite Gauss-Legendre
quadrature of their definitions instead.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

from .fdas_oracle import rho

__all__ = ["rho_moments_quad", "rho_derivs", "refine_window", "refine_power", "refine_spec_grad",
           "refine", "refine_starts", "ETA_R", "ETA_Z"]

ETA_R = 3.0 / (2.0 * math.pi ** 2)
ETA_Z = 90.0 / math.pi ** 2


def rho_moments_quad(q, z: float, order: int = 16):
    """(I0 = rho, I1, I2) with I_n = int_0^1 u^n exp(2 pi i [q u + z (u^2 - u)/2]) du, by
    composite Gauss-Legendre quadrature; panels turn the phase by at most ~1 rad."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    z = float(z)
    xg, wg = np.polynomial.legendre.leggauss(order)
    npan = int(math.ceil(2.0 * math.pi * (float(np.max(np.abs(q))) + abs(z) / 2.0 + 1.0))) + 4
    h = 1.0 / npan
    u = (np.arange(npan)[:, None] * h + 0.5 * h * (xg[None, :] + 1.0)).ravel()
    w = np.tile(0.5 * h * wg, npan)
    ph = 2.0 * np.pi * (q[:, None] * u[None, :] + z * (u * u - u)[None, :] * 0.5)
    e = np.exp(1j * ph) * w[None, :]
    return e.sum(axis=1), (e * u[None, :]).sum(axis=1), (e * (u * u)[None, :]).sum(axis=1)


def rho_derivs(q, z: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(rho, d rho/dq, d rho/dz) at offsets q (array) and drift z."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    z = float(z)
    # the identities lose ~(q/z)^2 ulps to cancellation: quadrature below that
    if abs(z) < max(1.0, float(np.max(np.abs(q))) / 16.0):
        r0, i1, i2 = rho_moments_quad(q, z)
    else:
        r0 = np.asarray(rho(q, z))
        e = np.exp(2j * np.pi * q)
        i1 = ((e - 1.0) / (2j * np.pi) - (q - z / 2.0) * r0) / z
        i2 = ((e - r0) / (2j * np.pi) - (q - z / 2.0) * i1) / z
    return r0, 2j * np.pi * i1, 1j * np.pi * (i2 - i1)


def refine_window(z0: float, dz: float, K: int = 16) -> int:
    """Window half-width M = ceil((|z0| + 2 dz)/2) + K + 1."""
    return int(math.ceil((abs(float(z0)) + 2.0 * float(dz)) / 2.0)) + int(K) + 1


def _window(Ah: np.ndarray, k0: int, M: int):
    """Bins k0-M..k0+M and their spectrum values (zero outside bins 1..len(Ah)-2)."""
    ks = np.arange(k0 - M, k0 + M + 1)
    nb = Ah.shape[0] - 1            # Ah holds bins 0..N/2
    ok = (ks >= 1) & (ks <= nb - 1)
    a = np.zeros(ks.shape, dtype=np.complex128)
    a[ok] = Ah[ks[ok]]
    return ks, a


def refine_power(Ah: np.ndarray, r: float, z: float, k0: int, M: int):
    """(P, dP/dr, dP/dz, c) of the refinement objective at (r, z), window (k0, M)."""
    ks, a = _window(Ah, k0, M)
    r0, dq, dzr = rho_derivs(float(r) - ks, z)
    c = np.sum(a * np.conj(r0))
    dcr = np.sum(a * np.conj(dq))
    dcz = np.sum(a * np.conj(dzr))
    P = float(abs(c) ** 2)
    return P, float(2.0 * np.real(np.conj(c) * dcr)), float(2.0 * np.real(np.conj(c) * dcz)), complex(c)


def refine_spec_grad(Ah: np.ndarray, r: float, z: float, k0: int, M: int):
    """(bins, g): g_k = dP/d Re(A^_k) + i dP/d Im(A^_k) = 2 c rho(r - k, z) over the window
    (zero for bins outside 1..N/2-1, which the objective does not read)."""
    ks, a = _window(Ah, k0, M)
    r0 = rho_derivs(float(r) - ks, z)[0]
    c = np.sum(a * np.conj(r0))
    g = 2.0 * c * r0
    nb = Ah.shape[0] - 1
    g[(ks < 1) | (ks > nb - 1)] = 0.0
    return ks, g


def refine(Ah: np.ndarray, r0: float, z0: float, dz: float, K: int = 16, iters: int = 20):
    """Ascent of the refinement objective from (r0, z0); returns (r, z, P) after iters steps."""
    k0 = int(math.floor(float(r0) + 0.5))
    M = refine_window(z0, dz, K)
    r, z = float(r0), float(z0)
    for _ in range(iters):
        P, gr, gz, _ = refine_power(Ah, r, z, k0, M)
        if not P > 0.0:
            break
        r = min(max(r + ETA_R * gr / P, r0 - 1.0), r0 + 1.0)
        z = min(max(z + ETA_Z * gz / P, z0 - 2.0 * dz), z0 + 2.0 * dz)
    P, _, _, _ = refine_power(Ah, r, z, k0, M)
    return r, z, P


def refine_starts(pl: np.ndarray, rlo: int, Z: int, count: int):
    """Start points: the count largest local maxima of a stage-1 plane on its integer-r
    cells (even R), each at least as large as its 8 neighbours on that sub-grid (R +- 2,
    Zq +- 1; ties go to the first in (R, Zq) order), as (R, Zq) pairs in decreasing
    power. pl: [NZ][NR], column c is R = c + 2 rlo."""
    NZ, NR = pl.shape
    sub = pl[:, 0::2]                   # R = 2 rlo + 2 j: integer r
    ns = sub.shape[1]
    pad = np.full((NZ + 2, ns + 2), -np.inf)
    pad[1:-1, 1:-1] = sub
    ismax = np.ones(sub.shape, dtype=bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = pad[1 + dy:1 + dy + NZ, 1 + dx:1 + dx + ns]
            earlier = (dx < 0) or (dx == 0 and dy < 0)
            ismax &= (sub > nb) if earlier else (sub >= nb)
    zi, ji = np.nonzero(ismax)
    vals = sub[zi, ji]
    order = np.lexsort((zi, ji, -vals))[:count]
    return [(int(2 * rlo + 2 * ji[i]), int(zi[i] - Z)) for i in order]
