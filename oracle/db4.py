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
  alternating sequence;
* a few square Newton steps on the N orthonormality and N moment equations follow in
  80-digit decimal arithmetic, because at N > 10 the moments (k^p up to 31^15 at N = 16)
  leave the double-precision polish about 1e-12 short; the result is then rounded once
  to double.

Time order follows eq. (9) of the paper, y_low[k] = sum_n x[n] h[2k - n].
"""
from __future__ import annotations

from decimal import Decimal, localcontext
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


def _newton_decimal(h: np.ndarray, N: int, steps: int = 4, digits: int = 80) -> np.ndarray:
    """Square Newton iteration on sum_k h_k h_{k+2m} = delta_m (m < N) and
    sum_k (-1)^k k^p h_k = 0 (p < N) in `digits`-digit decimals, Gaussian elimination with
    partial pivoting for each step."""
    n = len(h)
    with localcontext() as ctx:
        ctx.prec = digits
        x = [Decimal(float(v)) for v in h]
        alt = [Decimal(1 if k % 2 == 0 else -1) for k in range(n)]
        powk = [[Decimal(k ** p) for k in range(n)] for p in range(N)]
        for _ in range(steps):
            F, J = [], []
            for m in range(N):
                F.append(sum(x[k] * x[k + 2 * m] for k in range(n - 2 * m)) - (1 if m == 0 else 0))
                row = [Decimal(0)] * n
                for k in range(n - 2 * m):
                    row[k] += x[k + 2 * m]
                    row[k + 2 * m] += x[k]
                J.append(row)
            for p in range(N):
                F.append(sum(alt[k] * powk[p][k] * x[k] for k in range(n)))
                J.append([alt[k] * powk[p][k] for k in range(n)])
            A = [J[i][:] + [F[i]] for i in range(n)]
            for c in range(n):
                piv = max(range(c, n), key=lambda r: abs(A[r][c]))
                A[c], A[piv] = A[piv], A[c]
                for r in range(c + 1, n):
                    f = A[r][c] / A[c][c]
                    if f:
                        for q in range(c, n + 1):
                            A[r][q] -= f * A[c][q]
            dx = [Decimal(0)] * n
            for r in range(n - 1, -1, -1):
                t = A[r][n] - sum(A[r][q] * dx[q] for q in range(r + 1, n))
                dx[r] = t / A[r][r]
            x = [x[k] - dx[k] for k in range(n)]
        return np.array([float(v) for v in x])


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
        if N > 1:
            h = _newton_decimal(h, N)
    return h


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature-mirror high-pass g[m] = (-1)^m h[len-1-m] (used with eq. 8)."""
    n = len(h)
    return np.array([(-1.0) ** m * h[n - 1 - m] for m in range(n)])


DB4 = daubechies_lowpass(4)
