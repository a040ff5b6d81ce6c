"""Pins of the oracle's wavelet part against what the paper and the mathematics fix.

Sec. 3 (eqs. 8-9, Fig. 1) and Sec. 4 (Fig. 2, "until four samples are left") of the paper.
The filter is the 8-tap Daubechies filter (Daubechies 1992, Table 6.1 / Sec. 6.1).
"""
import os
from math import sqrt

import numpy as np
import pytest

import oracle
from oracle.db4 import daubechies_lowpass, highpass

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                rows.append(ln)
    return rows


def test_db4_matches_published_table():
    pub = np.array([float(r) for r in _load_golden("db4_daubechies1992.txt")])
    # printed to 12 decimals: agreement within half a unit of the last printed digit
    assert np.max(np.abs(oracle.DB4 - pub)) <= 5e-13


def test_db4_defining_conditions():
    h = oracle.DB4
    assert len(h) == 8
    assert abs(h.sum() - sqrt(2.0)) < 1e-15
    for m in range(4):
        s = np.dot(h[: 8 - 2 * m], h[2 * m:])
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-15
    g = highpass(h)
    k = np.arange(8, dtype=np.float64)
    for p in range(4):                       # four vanishing moments of the wavelet filter
        assert abs(np.sum(k ** p * g)) < 1e-12 * max(1.0, 7.0 ** p)


def test_db4_is_minimum_phase():
    # extremal phase: partial energies of h dominate those of every other spectral
    # factor; the reversed filter is the maximum-phase one
    h = oracle.DB4
    e, er = np.cumsum(h ** 2), np.cumsum(h[::-1] ** 2)
    assert np.all(e[:-1] >= er[:-1] - 1e-15)
    assert e[0] > er[0]


def test_daubechies_closed_forms():
    # N = 1 is the Haar filter; N = 2 has the closed form (1+r3, 3+r3, 3-r3, 1-r3)/(4 r2)
    assert np.allclose(daubechies_lowpass(1), [1 / sqrt(2)] * 2, atol=1e-16)
    r3 = sqrt(3.0)
    d2 = np.array([1 + r3, 3 + r3, 3 - r3, 1 - r3]) / (4 * sqrt(2.0))
    assert np.max(np.abs(daubechies_lowpass(2) - d2)) < 1e-15


def test_eq9_impulse_response_positions():
    # eq. (9): y_low[k] = sum_n x[n] h[2k - n].  A unit impulse at n0 puts h[2k - n0] at k.
    n, n0 = 32, 10
    x = np.zeros(n)
    x[n0] = 1.0
    a, d = oracle.dwt_level(x)
    expect = np.zeros(n // 2)
    for k in range(n // 2):
        m = 2 * k - n0
        if 0 <= m < 8:
            expect[k] = oracle.DB4[m]
    assert np.array_equal(a, expect)
    g = highpass(oracle.DB4)
    expect_d = np.zeros(n // 2)
    for k in range(n // 2):
        m = 2 * k - n0
        if 0 <= m < 8:
            expect_d[k] = g[m]
    assert np.array_equal(d, expect_d)


def _analysis_matrix(n):
    rows_a, rows_d = [], []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        a, d = oracle.dwt_level(e)
        rows_a.append(a)
        rows_d.append(d)
    return np.vstack([np.array(rows_a).T, np.array(rows_d).T])   # (n, n)


@pytest.mark.parametrize("n", [2, 4, 6, 8, 10, 16, 28, 64, 112, 224])
def test_one_level_is_orthogonal(n):
    Wm = _analysis_matrix(n)
    assert np.max(np.abs(Wm @ Wm.T - np.eye(n))) < 5e-15


def test_haar_reduction_at_length_two():
    x = np.array([0.3, -1.7])
    a, d = oracle.dwt_level(x)
    assert abs(a[0] - (x[0] + x[1]) / sqrt(2)) < 1e-15
    assert abs(d[0] - (x[0] - x[1]) / sqrt(2)) < 1e-15


@pytest.mark.parametrize("n,levels", [(224, 5), (64, 4), (128, 7), (96, 5)])
def test_perfect_reconstruction_and_energy(n, levels):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n)
    c = oracle.dwt_full(x, levels)
    assert abs(np.sum(c ** 2) - np.sum(x ** 2)) < 1e-12 * np.sum(x ** 2)
    xr = oracle.idwt_full(c, levels)
    assert np.max(np.abs(xr - x)) < 1e-13


def test_approx_part_of_full_transform():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 224)).astype(np.float32)
    a = oracle.dwt_approx(x, 5)
    for p in range(5):
        c = oracle.dwt_full(x[p].astype(np.float64), 5)
        assert np.array_equal(a[p], c[:7])


@pytest.mark.parametrize("L,levels", [(224, 6), (189, 5), (64, 4), (100, 5), (7, 2)])
def test_constant_signal(L, levels):
    # a constant c stays constant through the odd-length extension, and every level
    # multiplies it by sum(h) = sqrt(2)
    c = 0.75
    a = oracle.dwt_approx(np.full((1, L), c, dtype=np.float32), levels)[0]
    assert np.allclose(a, c * 2 ** (levels / 2), rtol=1e-14)
    _, d = oracle.dwt_level(np.full(L, c))
    assert np.max(np.abs(d)) < 1e-14


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_polynomials_have_no_interior_details(p):
    n = 64
    x = (np.arange(n, dtype=np.float64) / n) ** p
    _, d = oracle.dwt_level(x)
    # details whose 8-tap support does not wrap around (2k - 7 >= 0) vanish
    assert np.max(np.abs(d[4:])) < 1e-13


def test_odd_length_extends_by_last_sample():
    x = np.array([1.0, -2.0, 0.5])
    a3, d3 = oracle.dwt_level(x)
    a4, d4 = oracle.dwt_level(np.array([1.0, -2.0, 0.5, 0.5]))
    assert len(a3) == 2 and np.array_equal(a3, a4) and np.array_equal(d3, d4)


def test_fig2_lengths_and_level_rule():
    for row in _load_golden("fig2_lengths.txt"):
        L, lv, alen, dl = row.split()
        L, lv, alen = int(L), int(lv), int(alen)
        dls = [int(v) for v in dl.split(",")]
        assert oracle.dwt_out_len(L, lv) == alen
        c = oracle.dwt_full(np.arange(L, dtype=np.float64), lv)
        assert len(c) == alen + sum(dls)
    # "until four samples are left"
    assert oracle.levels_for(64) == 4 and oracle.dwt_out_len(64, 4) == 4
    assert oracle.levels_for(224) == 6 and oracle.dwt_out_len(224, 6) == 4
    assert oracle.levels_for(189) == 5 and oracle.dwt_out_len(189, 5) == 6


def test_out_len_rules():
    assert oracle.dwt_out_len(224, 0) == 224
    assert [oracle.dwt_out_len(224, j) for j in range(1, 7)] == [112, 56, 28, 14, 7, 4]
    assert oracle.dwt_out_len(189, 1) == 95
    assert oracle.dwt_out_len(1, 1) == -1
    assert oracle.dwt_out_len(3, 2) == 1
    assert oracle.dwt_out_len(3, 3) == -1


# ---------------------------------------------------------------------------------------
# Other Daubechies orders (Fig. 2 uses a 16-vanishing-moment filter) and the full
# transform on odd-length chains
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 3, 4, 6, 8, 10, 12, 16])
def test_daubechies_family_defining_conditions(N):
    """The defining equations hold to rounding and the filter has extremal (minimum)
    phase.  Together they determine the filter."""
    h = daubechies_lowpass(N)
    n = 2 * N
    tol = 1e-14
    assert len(h) == n
    assert abs(h.sum() - sqrt(2.0)) < tol
    for m in range(N):
        s = float(np.dot(h[: n - 2 * m], h[2 * m:]))
        assert abs(s - (1.0 if m == 0 else 0.0)) < tol, m
    g = highpass(h)
    k = np.arange(n, dtype=np.float64)
    for p in range(N):
        assert abs(np.sum(k ** p * g)) < tol * max(1.0, np.abs(k ** p * g).sum()), p
    if N > 1:
        # sum h[n] w^n (w = 1/z) has an N-fold zero at w = -1, which rounding splits into a
        # small cluster, and N - 1 further zeros, all outside the unit circle
        r = np.roots(h[::-1])
        far, near = r[np.abs(r) > 1.3], r[np.abs(r) <= 1.3]
        assert len(far) == N - 1 and len(near) == N
        assert np.max(np.abs(near + 1.0)) < 0.25


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("n,levels", [(224, 5), (64, 2), (96, 5)])
def test_family_orthogonality_on_even_chains(N, n, levels):
    h = daubechies_lowpass(N)
    rng = np.random.default_rng(N * 100 + n)
    x = rng.standard_normal(n)
    c = oracle.dwt_full(x, levels, h)
    assert len(c) == n
    assert abs(np.sum(c ** 2) - np.sum(x ** 2)) < 1e-12 * np.sum(x ** 2)
    assert np.max(np.abs(oracle.idwt_full(c, levels, h) - x)) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("n,levels", [(224, 6), (189, 5), (7, 2), (33, 5), (100, 5)])
def test_full_transform_odd_chains_reconstruct(N, n, levels):
    """Odd level inputs are extended by their last sample (the approximation's rule applied
    to both branches), so the transform is injective and the inverse recovers x."""
    h = daubechies_lowpass(N)
    rng = np.random.default_rng(N + n + levels)
    x = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    c = oracle.dwt_full(x, levels, h)
    lens, m = [], n
    for _ in range(levels):
        m = (m + 1) // 2
        lens.append(m)
    assert len(c) == lens[-1] + sum(lens) == oracle.dwt_full_len(n, levels)
    assert np.array_equal(c[:lens[-1]], oracle.dwt_approx(x[None, :].astype(np.float32), levels, h)[0])
    xr = oracle.idwt_full(c, levels, h, n=n)
    assert np.max(np.abs(xr - x)) < 1e-12


def test_full_transform_odd_level_equals_extended_even_level():
    # one level of an odd signal = one level of the signal with its last sample repeated,
    # whose energy is preserved (orthogonal level)
    rng = np.random.default_rng(5)
    for N in (1, 4, 16):
        h = daubechies_lowpass(N)
        x = rng.standard_normal(37)
        xe = np.concatenate([x, x[-1:]])
        c = oracle.dwt_full(x, 1, h)
        ce = oracle.dwt_full(xe, 1, h)
        assert np.array_equal(c, ce)
        assert abs(np.sum(ce ** 2) - np.sum(xe ** 2)) < 1e-12 * np.sum(xe ** 2)


def test_full_transform_layout_and_haar_closed_form():
    # Haar (h = [1, 1]/sqrt 2, g = [1, -1]/sqrt 2) with eq. (9)'s periodic index pairs
    # x[2k] with x[2k - 1]: level 1 on [x0..x3] gives a1 = ((x0+x3), (x2+x1))/sqrt 2 and
    # d1 = ((x0-x3), (x2-x1))/sqrt 2; level 2 gives a2 = (x0+x1+x2+x3)/2 and
    # d2 = (a1[0] - a1[1])/sqrt 2.  Output order [a2 d2 d1].
    x = np.array([1.0, 2.0, 4.0, 8.0])
    c = oracle.dwt_full(x, 2, daubechies_lowpass(1))
    r2 = sqrt(2.0)
    want = [7.5, (x[0] + x[3] - x[2] - x[1]) / 2, (x[0] - x[3]) / r2, (x[2] - x[1]) / r2]
    assert np.allclose(c, want, rtol=0, atol=1e-14)


def test_full_cube_forms_match_signal_forms():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((3, 4, 45)).astype(np.float32)
    h = daubechies_lowpass(8)
    c = oracle.dwt_full_cube(x, 3, h)
    assert c.shape == (3, 4, oracle.dwt_full_len(45, 3))
    for p in range(12):
        v = x.reshape(12, 45)[p].astype(np.float64)
        assert np.array_equal(c.reshape(12, -1)[p], oracle.dwt_full(v, 3, h))
    xr = oracle.idwt_full_cube(c.astype(np.float32), 45, 3, h)
    assert xr.shape == x.shape and np.max(np.abs(xr - x)) < 1e-5
