"""Pins of the oracle's Jacobi eigensolver and DWEST (Sec. 2.2, eqs. 2-4).

LAPACK (numpy.linalg.eigh) is the independent reference for the eigen-decomposition.
DWEST has these invariances: orthogonal maps of the spectra, shifts, and scaling by c,
which multiplies the score by |c|.
"""
import numpy as np
import pytest

import oracle
from paper_1201_2025_amd import synth


@pytest.mark.parametrize("n", [1, 2, 3, 7, 14, 28])
def test_jacobi_against_lapack(n):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    A = M + M.T
    ev, V, sweeps = oracle.jacobi_eig(A)
    assert np.allclose(np.sort(ev), np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
    assert np.allclose(A @ V, V * ev, atol=1e-12 * np.abs(A).max())
    assert sweeps < 20


def _brute_dwest(x, inner, outer):
    H, W, L = x.shape
    ro, ri = outer // 2, inner // 2
    yy, xx = np.mgrid[0:H, 0:W]
    score = np.zeros(H * W)
    literal = np.zeros(H * W)
    npos = np.zeros(H * W, dtype=int)
    for p in range(H * W):
        py, px = divmod(p, W)
        ob = (np.abs(yy - py) <= ro) & (np.abs(xx - px) <= ro)
        ib = (np.abs(yy - py) <= ri) & (np.abs(xx - px) <= ri)
        A, I = x[ob & ~ib], x[ib]
        Cd = np.cov(I.T, bias=True).reshape(L, L) - np.cov(A.T, bias=True).reshape(L, L)
        md = I.mean(0) - A.mean(0)
        e, V = np.linalg.eigh(Cd)
        keep = e > 1e-12 * np.abs(e).max()
        proj = V[:, keep].T @ md
        score[p] = np.linalg.norm(proj)
        # eq. (4) summed over the positive eigenvectors, each signed so that its
        # projection is non-negative: the sum of the absolute projections
        literal[p] = np.abs(proj).sum()
        npos[p] = keep.sum()
    return score, literal, npos


@pytest.mark.parametrize("H,W,L,inner,outer", [(7, 6, 3, 3, 5), (6, 8, 5, 3, 7), (5, 5, 2, 1, 3)])
def test_dwest_bruteforce(H, W, L, inner, outer):
    x = synth.random_cube(H + W + L, H, W, L).astype(np.float64)
    s, lit, npos = oracle.dwest(x, inner, outer)
    bs, bl, bn = _brute_dwest(x, inner, outer)
    assert np.allclose(s, bs, rtol=1e-9, atol=1e-12)
    assert np.allclose(lit, bl, rtol=1e-9, atol=1e-12)
    assert np.array_equal(npos, bn)


def test_dwest_literal_bruteforce_larger_bands():
    """The literal score against LAPACK's eigenvectors on a scene cube with L' = 9 bands
    and a 3 x 3 / 9 x 9 window, where several eigenvalues are positive per pixel."""
    s = synth.make_scene(77, 12, 11, 9, K=3, n_single=2)
    x = s.cube.astype(np.float64)
    sc, lit, npos = oracle.dwest(x, 3, 9)
    bs, bl, bn = _brute_dwest(x, 3, 9)
    assert np.array_equal(npos, bn)
    assert (npos >= 2).mean() > 0.5
    assert np.allclose(sc, bs, rtol=1e-8, atol=1e-12 * np.abs(bs).max())
    assert np.allclose(lit, bl, rtol=1e-8, atol=1e-12 * np.abs(bl).max())


def test_dwest_invariances_and_bounds():
    H, W, L = 9, 8, 4
    x = synth.random_cube(21, H, W, L).astype(np.float64)
    s, lit, npos = oracle.dwest(x, 3, 7)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((L, L)))
    s2, _, n2 = oracle.dwest(x @ Q.T + 5.0, 3, 7)
    assert np.allclose(s, s2, rtol=1e-8, atol=1e-12) and np.array_equal(npos, n2)
    s3, lit3, _ = oracle.dwest(-2.0 * x, 3, 7)
    assert np.allclose(s3, 2.0 * s, rtol=1e-9) and np.allclose(lit3, 2.0 * lit, rtol=1e-9)
    # at most rank(C_inner) <= n_inner - 1 positive eigenvalues; l1 >= l2 >= l1/sqrt(k)
    assert np.all(npos <= 8)
    assert np.all(lit >= s - 1e-12)
    assert np.all(lit <= np.sqrt(np.maximum(npos, 1)) * s + 1e-12)


def test_dwest_zero_when_windows_match():
    x = np.full((5, 5, 3), 1.25)
    s, lit, npos = oracle.dwest(x, 3, 5)
    assert np.all(s == 0) and np.all(lit == 0) and np.all(npos == 0)
