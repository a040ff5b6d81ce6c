"""Daubechies low-pass filters derived from their definition (oracle side).

Test infrastructure only.

The paper applies a "Daubechies4" wavelet (abstract; Sec. 4).  It is read here as the
8-tap Daubechies filter with 4 vanishing moments.  The filter is not copied from a table.
It is constructed the way Daubechies defines it (Ten Lectures on Wavelets, 1992, Sec. 6.1):

* |m0(xi)|^2 = cos^{2N}(xi/2) P(sin^2(xi/2)), with P(y) = sum_{k<N} C(N-1+k, k) y^k;
* spectral factorisation of P keeps, for every root pair (z, 1/z), the root inside the
  unit circle.  This is the minimum-phase ("extremal phase") choice;
* h is normalised to sum(h) = sqrt(2);
* a Gauss-Newton polish is then applied on the defining equations.  These are
  orthonormality of even shifts, sum(h) = sqrt(2), and N vanishing moments of the
  alternating sequence.

Time order follows eq. (9) of the paper, y_low[k] = sum_n x[n] h[2k - n].
"""
from __future__ import annotations

from math import comb, sqrt

import numpy as np


def _defining_equations(h: np.ndarray, N: int) -> np.ndarray:
    n = len(h)
    eqs = [h.sum() - sqrt(2.0)]
    for m in range(N):                         # sum_k h_k h_{k+2m} = delta_m
        eqs.append(float(np.dot(h[: n - 2 * m], h[2 * m:])) - (1.0 if m == 0 else 0.0))
    k = np.arange(n, dtype=np.float64)
    alt = (-1.0) ** k
    for p in range(N):                         # sum_k (-1)^k k^p h_k = 0
        eqs.append(float(np.sum(alt * k ** p * h)))
    return np.array(eqs)


def _jacobian(h: np.ndarray, N: int) -> np.ndarray:
    n = len(h)
    rows = [np.ones(n)]
    for m in range(N):
        r = np.zeros(n)
        if m == 0:
            r = 2.0 * h
        else:
            r[: n - 2 * m] += h[2 * m:]
            r[2 * m:] += h[: n - 2 * m]
        rows.append(r)
    k = np.arange(n, dtype=np.float64)
    for p in range(N):
        rows.append((-1.0) ** k * k ** p)
    return np.array(rows)


def daubechies_lowpass(N: int = 4, polish: bool = True) -> np.ndarray:
    """2N-tap minimum-phase Daubechies scaling filter with N vanishing moments."""
    if N < 1:
        raise ValueError("N >= 1")
    # P(y) coefficients, highest power first for numpy.roots
    P = [comb(N - 1 + k, k) for k in range(N)][::-1]
    poly = np.poly1d([1.0])                   # product over roots of (1 - z_r w), w = 1/z
    for y in (np.roots(P) if N > 1 else []):
        # y = (2 - z - 1/z)/4  <=>  z^2 - (2 - 4y) z + 1 = 0
        zs = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        z = zs[np.argmin(np.abs(zs))]          # inside the unit circle: minimum phase
        poly = poly * np.poly1d([-z, 1.0])     # (1 - z w) written highest power first
    binom = np.poly1d([1.0])
    for _ in range(N):
        binom = binom * np.poly1d([1.0, 1.0])  # (1 + w)^N
    full = binom * poly
    # poly1d stores highest power first; h[n] multiplies w^n
    h = np.real(full.coeffs[::-1]).astype(np.float64)
    h *= sqrt(2.0) / h.sum()
    if polish:
        for _ in range(8):
            F = _defining_equations(h, N)
            J = _jacobian(h, N)
            step, *_ = np.linalg.lstsq(J, F, rcond=None)
            h = h - step
            if np.max(np.abs(step)) < 1e-17:
                break
    return h


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature-mirror high-pass g[m] = (-1)^m h[len-1-m] (used with eq. 8)."""
    n = len(h)
    return np.array([(-1.0) ** m * h[n - 1 - m] for m in range(n)])


DB4 = daubechies_lowpass(4)
