"""Pins of the oracle's window statistics, LRX (eq. 1) and DWRX (eq. 5).

The pins are closed forms, invariances and an independent numpy brute force.  The
global RX mean is L', the leave-one-out identity is stated below, and RX is unchanged
by affine and orthogonal maps.
"""
import numpy as np
import pytest

import oracle
from paper_1201_2025_amd import synth


def _cube(seed, H, W, L, scale=1.0):
    return synth.random_cube(seed, H, W, L, scale).astype(np.float64)


def test_global_rx_mean_equals_band_count():
    # whole-image window, no guard window, no loading: sum_i (x_i-mu)^T C^-1 (x_i-mu)
    # = tr(C^-1 * N C) = N L'  with the 1/N covariance
    H, W, L = 9, 11, 5
    x = _cube(1, H, W, L)
    outer = 2 * max(H, W) + 1
    lrx, _ = oracle.lrx_dwrx(x, 0, outer, load_rel=0.0)
    assert abs(lrx.mean() - L) < 1e-10


def test_global_rx_mean_with_loading():
    H, W, L = 8, 9, 4
    x = _cube(2, H, W, L)
    rel = 0.05
    lrx, _ = oracle.lrx_dwrx(x, 0, 2 * max(H, W) + 1, load_rel=rel)
    X = x.reshape(-1, L)
    C = np.cov(X.T, bias=True)
    e = np.linalg.eigvalsh(C)
    lam = rel * np.trace(C) / L
    assert abs(lrx.mean() - np.sum(e / (e + lam))) < 1e-10


def test_leave_one_out_identity():
    # inner = 1 removes the pixel itself from the whole-image background.  With N pixels
    # and global score D_i: LRX_i = N D_i / (N - 1 - D_i)  (Sherman-Morrison)
    H, W, L = 7, 8, 3
    x = _cube(3, H, W, L)
    N = H * W
    outer = 2 * max(H, W) + 1
    g, _ = oracle.lrx_dwrx(x, 0, outer, load_rel=0.0)
    loo, _ = oracle.lrx_dwrx(x, 1, outer, load_rel=0.0)
    assert np.allclose(loo, N * g / (N - 1 - g), rtol=1e-10)


def test_affine_invariance_without_loading():
    H, W, L = 10, 10, 4
    x = _cube(4, H, W, L)
    rng = np.random.default_rng(0)
    A = rng.standard_normal((L, L)) + 3 * np.eye(L)
    b = rng.standard_normal(L)
    y = x @ A.T + b
    for inner, outer in [(0, 5), (3, 7), (1, 9)]:
        l1, d1 = oracle.lrx_dwrx(x, inner, outer, load_rel=0.0)
        l2, d2 = oracle.lrx_dwrx(y, inner, outer, load_rel=0.0)
        assert np.allclose(l1, l2, rtol=1e-8)
        if inner:
            assert np.allclose(d1, d2, rtol=1e-8, atol=1e-12)


def test_scale_shift_invariance_with_relative_loading():
    x = _cube(5, 12, 9, 6)
    l1, d1 = oracle.lrx_dwrx(x, 3, 7, load_rel=1e-3)
    l2, d2 = oracle.lrx_dwrx(-3.5 * x + 10.0, 3, 7, load_rel=1e-3)
    assert np.allclose(l1, l2, rtol=1e-9) and np.allclose(d1, d2, rtol=1e-9)


def test_rx_invariant_under_full_orthogonal_dwt():
    # the full DWT (eqs. 8-9 iterated, all coefficients kept) is an orthogonal map of each
    # spectrum, and tr(C) is orthogonally invariant, so LRX/DWRX with relative loading
    # are unchanged
    H, W, L, lv = 9, 10, 16, 3
    x = _cube(6, H, W, L)
    c = np.stack([oracle.dwt_full(v, lv) for v in x.reshape(-1, L)]).reshape(H, W, L)
    l1, d1 = oracle.lrx_dwrx(x, 3, 7, load_rel=1e-4)
    l2, d2 = oracle.lrx_dwrx(c, 3, 7, load_rel=1e-4)
    assert np.allclose(l1, l2, rtol=1e-9) and np.allclose(d1, d2, rtol=1e-9)


def test_constant_cube_scores_zero():
    x = np.full((6, 7, 3), 2.5)
    l, d = oracle.lrx_dwrx(x, 3, 5, load_rel=1e-6)
    assert np.all(l == 0.0) and np.all(d == 0.0)


def test_loading_floor_and_value():
    C = np.diag([1.0, 2.0, 3.0])
    assert oracle.loading(C, 1e-6) == pytest.approx(2e-6, rel=1e-15)
    assert oracle.loading(np.zeros((3, 3)), 1e-6) == 1e-30
    assert oracle.loading(C, 0.0) == 1e-30


def test_cholesky_against_numpy():
    rng = np.random.default_rng(11)
    for n in (1, 2, 5, 17):
        M = rng.standard_normal((n, n + 3))
        A = M @ M.T
        Lf = oracle.cholesky(A)
        assert np.allclose(Lf, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    assert oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]])) is None


def _brute(x, inner, outer, load_rel):
    """Independent numpy gather: masks over the clipped window, np.cov, np.linalg.solve."""
    H, W, L = x.shape
    ro, ri = outer // 2, inner // 2
    lrx = np.zeros((H, W))
    dwrx = np.zeros((H, W))
    yy, xx = np.mgrid[0:H, 0:W]
    for py in range(H):
        for px in range(W):
            ob = (np.abs(yy - py) <= ro) & (np.abs(xx - px) <= ro)
            ib = (np.abs(yy - py) <= ri) & (np.abs(xx - px) <= ri) if inner else np.zeros_like(ob)
            A = x[ob & ~ib]
            Cn = np.cov(A.T, bias=True).reshape(L, L)
            mu = A.mean(0)
            lam = max(load_rel * np.trace(Cn) / L, 1e-30)
            M = Cn + lam * np.eye(L)
            d = x[py, px] - mu
            lrx[py, px] = d @ np.linalg.solve(M, d)
            if inner:
                m = x[ib].mean(0) - mu
                dwrx[py, px] = m @ np.linalg.solve(M, m)
    return lrx.ravel(), dwrx.ravel()


@pytest.mark.parametrize("H,W,L,inner,outer", [
    (6, 7, 3, 3, 5), (5, 9, 1, 1, 3), (8, 6, 4, 0, 5), (4, 4, 2, 3, 7), (9, 5, 5, 1, 9)])
def test_bruteforce_tiny_cubes(H, W, L, inner, outer):
    x = _cube(H * 100 + W, H, W, L)
    l, d = oracle.lrx_dwrx(x, inner, outer, load_rel=1e-2)
    bl, bd = _brute(x, inner, outer, 1e-2)
    assert np.allclose(l, bl, rtol=1e-9, atol=1e-12)
    if inner:
        assert np.allclose(d, bd, rtol=1e-9, atol=1e-12)


def test_window_stats_counts_at_border():
    x = _cube(9, 10, 12, 2)
    n_a, mu, C, n_in, mi, Ci = oracle.window_stats(x, 3, 7, 0, 0)
    assert n_a == 4 * 4 - 2 * 2 and n_in == 4
    n_a, mu, C, n_in, mi, Ci = oracle.window_stats(x, 3, 7, 5, 6)
    assert n_a == 49 - 9 and n_in == 9
    win = x[2:9, 3:10]
    ring = np.ones((7, 7), dtype=bool)
    ring[2:5, 2:5] = False
    assert np.allclose(mu, win[ring].mean(0), rtol=1e-14)
    assert np.allclose(C, np.cov(win[ring].T, bias=True), rtol=1e-12)
    assert np.allclose(mi, win[~ring].mean(0), rtol=1e-14)


def test_dwt_then_lrx_on_generated_scene():
    # sanity on the generator: with the DWT reduction the implanted targets stand out
    cfg = synth.CONFIGS["small_64x64x224"]
    s = synth.make_scene(cfg["seed"], cfg["H"], cfg["W"], cfg["L"], K=cfg["K"],
                         n_single=cfg["n_single"], n_blob=cfg["n_blob"])
    a = oracle.dwt_approx(s.cube, cfg["levels"])
    l, _ = oracle.lrx_dwrx(a, cfg["inner"], cfg["outer"], cfg["load_rel"])
    assert oracle.auc(l, s.truth) > 0.95


# ---------------------------------------------------------------------------------------
# Global RX (Sec. 2.1, eq. 1 with every pixel as background)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("rel", [0.0, 1e-6, 0.05])
def test_global_rx_is_whole_image_window_lrx(rel):
    # the global background is the local one with a window covering the image and no
    # guard window: two independent routes in the oracle
    H, W, L = 7, 9, 4
    x = _cube(31, H, W, L)
    g = oracle.global_rx(x, rel)
    lrx, _ = oracle.lrx_dwrx(x, 0, 2 * max(H, W) + 1, load_rel=rel)
    assert np.allclose(g, lrx, rtol=1e-11, atol=1e-13)


def test_global_rx_mean_and_loading_closed_forms():
    H, W, L = 40, 37, 9
    x = _cube(32, H, W, L, scale=3.0) + 5.0
    assert abs(oracle.global_rx(x, 0.0).mean() - L) < 1e-10
    rel = 0.02
    X = x.reshape(-1, L)
    C = np.cov(X.T, bias=True)
    e = np.linalg.eigvalsh(C)
    lam = rel * np.trace(C) / L
    assert abs(oracle.global_rx(x, rel).mean() - np.sum(e / (e + lam))) < 1e-10


def test_global_rx_stats_and_leave_one_out():
    H, W, L = 12, 10, 5
    x = _cube(33, H, W, L)
    s, mu, C = oracle.global_rx(x, 0.0, stats=True)
    X = x.reshape(-1, L)
    assert np.allclose(mu, X.mean(0), rtol=1e-14, atol=1e-15)
    assert np.allclose(C, np.cov(X.T, bias=True), rtol=1e-13, atol=1e-15)
    N = H * W
    loo, _ = oracle.lrx_dwrx(x, 1, 2 * max(H, W) + 1, load_rel=0.0)
    assert np.allclose(loo, N * s / (N - 1 - s), rtol=1e-10)


def test_global_rx_affine_invariance_and_subset():
    H, W, L = 15, 14, 6
    x = _cube(34, H, W, L)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((L, L)) + 2 * np.eye(L)
    y = x @ A.T + rng.standard_normal(L)
    g1, g2 = oracle.global_rx(x, 0.0), oracle.global_rx(y, 0.0)
    assert np.allclose(g1, g2, rtol=1e-8)
    idx = np.array([0, 17, H * W - 1, 17])
    assert np.array_equal(oracle.global_rx(x, 1e-6, idx=idx), oracle.global_rx(x, 1e-6)[idx])


def test_sample_rounding_matches_library_conversions():
    """The reduced-precision roundings of the oracle against numpy's binary32 and binary16
    and torch's bfloat16 conversions (each from binary32, round to nearest even), on
    ordinary values, ties, subnormals, overflow and signed zero."""
    import torch
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-9, 6, 4000),
                        [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.0, 65520.0, 1e6, -1e6, 2.0 ** -24,
                         2.0 ** -25, 3 * 2.0 ** -26, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9,
                         1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -12, 1e-40, np.inf, -np.inf]])
    f32 = v.astype(np.float32)
    assert np.array_equal(oracle.round_samples(v, "fp32"), f32.astype(np.float64))
    with np.errstate(over="ignore"):
        want16 = f32.astype(np.float16).astype(np.float64)
    got16 = oracle.round_samples(v, "fp16")
    assert np.array_equal(np.signbit(got16), np.signbit(want16))
    assert np.array_equal(got16, want16)
    wantbf = torch.from_numpy(f32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_samples(v, "bf16"), wantbf)
    assert np.array_equal(oracle.round_samples(v, None), v)


def test_rounded_statistics_reduce_to_exact_on_representable_data():
    """Data whose centred samples are exactly representable in bfloat16 (small integers on a
    window whose mean is an integer) gives the same LRX with and without rounding."""
    x = np.zeros((9, 9, 3))
    rng = np.random.default_rng(4)
    x[:] = rng.integers(-4, 5, size=(9, 9, 3))
    # single pixel whose 3 x 3 annulus (inner 1) mean is integral: make it so by construction
    idx = np.array([4 * 9 + 4])
    ann = [(4 + dy) * 9 + 4 + dx for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]
    flat = x.reshape(-1, 3)
    flat[ann[-1]] += (8 - flat[ann].sum(axis=0) % 8) % 8   # annulus sums divisible by 8
    for r in ("fp32", "bf16", "fp16"):
        a = oracle.lrx_dwrx(x, 1, 3, 1e-6, idx=idx, want=("lrx",))[0]
        b = oracle.lrx_dwrx(x, 1, 3, 1e-6, idx=idx, want=("lrx",), rounding=r)[0]
        assert np.array_equal(a, b)
