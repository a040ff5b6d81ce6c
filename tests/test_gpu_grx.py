"""GPU parity of hsad_global_rx (eq. 1 of Sec. 2.1 with every pixel of the image as the
background) against the FP64 oracle, plus the closed forms that pin it independently:
  * without loading the mean score over the image is exactly L' (1/N sum_p d_p^T C^-1 d_p
    = tr(C^-1 C));
  * with loading lambda it is sum_i e_i / (e_i + lambda) over the eigenvalues e_i of C;
  * leave-one-out: LRX with a window covering the whole image and only the pixel itself
    excluded (inner = 1, no loading) equals N D / (N - 1 - D), D the global score.  The
    two sides run different kernels (box sums + register Cholesky against the global
    Gram + blocked factorisation).
Scores: elementwise relative error <= 1e-3 with a floor of 1e-3 * median (as LRX).
"""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import err_summary, sample_pixels, scene, score_rel_err

pytestmark = pytest.mark.gpu


def _cube(seed, H, W, Lp, L=224):
    lv = [j for j in range(12) if oracle.dwt_out_len(L, j) == Lp]
    if not lv:   # not a level of 224 bands: a raw cube of Lp bands
        return scene(seed, H, W, Lp).cube
    s = scene(seed, H, W, L)
    return s.cube if lv[0] == 0 else oracle.dwt_approx(s.cube, lv[0]).astype(np.float32)


def _gpu(x, load_rel=1e-6, stats=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    r = hs.hsad_global_rx(t, load_rel, stats=stats)
    torch.cuda.synchronize()
    if stats:
        return tuple(a.cpu().numpy() for a in r)
    return r.cpu().numpy()


# ragged tile counts (L' = 4, 14, 56, 100, 224 pad to 16, 16, 64, 112, 224), full band
# with fewer bands than pixels, and the 256-band maximum
CASES = [(37, 29, 4), (64, 64, 14), (48, 40, 56), (40, 33, 100), (32, 32, 224), (24, 20, 7), (1, 64, 4)]


@pytest.mark.parametrize("H,W,Lp", CASES)
@pytest.mark.parametrize("load_rel", [1e-6, 0.0])
def test_global_rx_matches_oracle(H, W, Lp, load_rel):
    print("grx case H=%d W=%d Lp=%d load=%g" % (H, W, Lp, load_rel), flush=True)
    x = _cube(2100 + Lp, H, W, Lp)
    if H * W <= Lp and load_rel == 0.0:
        pytest.skip("singular covariance without loading")
    g, gm, gc = _gpu(x, load_rel, stats=True)
    r, rm, rc = oracle.global_rx(x.astype(np.float64), load_rel, stats=True)
    assert np.max(np.abs(gm - rm)) <= 1e-12 * max(1.0, np.max(np.abs(rm)))
    assert np.max(np.abs(gc - rc)) <= 1e-9 * np.max(np.abs(rc))
    assert np.array_equal(gc, gc.T)
    e = score_rel_err(g.ravel(), r)
    print("grx", H, W, Lp, load_rel, err_summary(e), flush=True)
    assert e.max() <= 1e-3


def test_global_rx_256_bands():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((40, 30, 256)).astype(np.float32) + rng.random(256).astype(np.float32)
    g = _gpu(x, 1e-6)
    r = oracle.global_rx(x.astype(np.float64), 1e-6)
    assert score_rel_err(g.ravel(), r).max() <= 1e-3


@pytest.mark.parametrize("H,W,Lp", [(64, 48, 4), (50, 50, 28), (40, 40, 224)])
def test_mean_score_is_band_count(H, W, Lp):
    x = _cube(2200 + Lp, H, W, Lp).astype(np.float32)
    g = _gpu(x, 0.0).astype(np.float64)
    assert abs(g.mean() - Lp) <= 2e-4 * Lp
    lam_rel = 1e-3
    g2, _, C = _gpu(x, lam_rel, stats=True)
    ev = np.linalg.eigvalsh(C)
    lam = lam_rel * np.trace(C) / Lp
    want = float(np.sum(ev / (ev + lam)))
    assert abs(g2.astype(np.float64).mean() - want) <= 2e-4 * want


@pytest.mark.parametrize("H,W,Lp", [(32, 32, 4), (31, 27, 7), (32, 30, 14)])
def test_leave_one_out_identity(H, W, Lp):
    import torch
    x = _cube(2300 + Lp, H, W, Lp)
    D = _gpu(x, 0.0).astype(np.float64).ravel()
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    outer = 2 * max(H, W) - 1
    lrx, _ = hs.hsad_lrx_dwrx(t, 1, outer, 0.0, lrx=True, dwrx=False)
    torch.cuda.synchronize()
    lrx = lrx.cpu().numpy().astype(np.float64).ravel()
    N = H * W
    want = N * D / (N - 1 - D)
    err = score_rel_err(lrx, want)
    print("leave-one-out", H, W, Lp, err_summary(err), flush=True)
    assert err.max() <= 1e-3


def test_non_finite_gives_inf_everywhere():
    x = _cube(2400, 20, 20, 4).copy()
    x[3, 4, 1] = np.nan
    g = _gpu(x, 1e-6)
    assert np.all(np.isposinf(g))
    r = oracle.global_rx(x.astype(np.float64), 1e-6)
    assert np.all(np.isposinf(r))


def test_deterministic():
    x = _cube(2500, 64, 64, 56)
    a = _gpu(x)
    b = _gpu(x)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("levels", [6, 0])
def test_full_size_sampled(levels):
    """512 x 512 x 224 cube at L' = 4 and at full band (L' = 224): the oracle computes the
    global statistics over all 262 144 pixels and scores a sample of them."""
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["cube_512x512x224"]
    print("grx full size levels=%d" % levels, flush=True)
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
    t = torch.from_numpy(s.cube).cuda()
    a = hs.hsad_dwt(t, levels) if levels else t
    g = hs.hsad_global_rx(a, 1e-6)
    torch.cuda.synchronize()
    g = g.cpu().numpy().ravel()
    x = oracle.dwt_approx(s.cube, levels) if levels else s.cube.astype(np.float64)
    idx = sample_pixels(c["H"], c["W"], 3000, seed=levels)
    r = oracle.global_rx(x, 1e-6, idx=idx)
    e = score_rel_err(g[idx], r)
    print("grx full size", levels, err_summary(e), flush=True)
    assert e.max() <= 1e-3
