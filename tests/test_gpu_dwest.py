"""GPU parity of hsad_dwest (Sec. 2.2, eqs. 2-4) against the FP64 oracle.

Scores (||V_P^T m_diff||_2), literal scores (sum_P |v_i^T m_diff|) and the number of
positive eigenvalues are compared.  The score bound is an elementwise relative error
<= 1e-3, with a floor of 1e-3 * median.  The positive-eigenvalue counts must match
exactly.  Every GPU eigensolver mode is covered (selected through an internal switch):
Householder tridiagonalisation + implicit QL over runs of pixels with the tridiagonal forms
in global columns, the same QL per chunk with LDS columns (the default picks one of the
two), and the cyclic Jacobi solver; the window statistics from box sums (the default where
supported) or from the matrix-core Gram.
"""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import err_summary, sample_pixels, scene, score_rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-3


# (solver switch, statistics: 0 box sums where supported / 1 matrix-core Gram)
SOLVERS = {"ql": (0, 0), "jacobi": (1, 0), "ql_chunk": (2, 0), "ql_runs": (3, 0), "ql_gram": (0, 1),
           "ql_runs_gram": (3, 1)}


@pytest.fixture(params=sorted(SOLVERS))
def solver(request):
    L_ = hs.lib()
    sv, st = SOLVERS[request.param]
    L_.hsad_internal_dwest_solver(sv)
    L_.hsad_internal_dwest_stats(st)
    yield request.param
    L_.hsad_internal_dwest_solver(0)
    L_.hsad_internal_dwest_stats(0)


def _gpu(x, inner, outer):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    s, lit, npos = hs.hsad_dwest(t, inner, outer)
    torch.cuda.synchronize()
    return s.cpu().numpy().ravel(), lit.cpu().numpy().ravel(), npos.cpu().numpy().ravel()


@pytest.mark.parametrize("H,W,levels,inner,outer", [
    (26, 21, 4, 3, 11), (17, 19, 3, 3, 11), (9, 10, 2, 3, 11), (20, 20, 6, 5, 13),
    (15, 33, 5, 1, 7), (6, 5, 4, 3, 5)])
def test_dwest_parity(H, W, levels, inner, outer, solver):
    s = scene(H * W + levels, H, W, 224)
    x = oracle.dwt_approx(s.cube, levels).astype(np.float32)
    gs, gl, gn = _gpu(x, inner, outer)
    rs, rl, rn = oracle.dwest(x.astype(np.float64), inner, outer)
    e = score_rel_err(gs, rs)
    el = score_rel_err(gl, rl)
    print("dwest", x.shape, inner, outer, "score", err_summary(e), "literal", err_summary(el),
          "npos mismatches", int((gn != rn).sum()), flush=True)
    assert np.array_equal(gn, rn)
    assert e.max() <= TOL
    assert el.max() <= TOL


@pytest.mark.parametrize("levels", [4, 3, 2])
def test_dwest_full_size_sampled(levels):
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["dwest_512x512x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"],
                         n_blob=c["n_blob"])
    t = torch.from_numpy(s.cube).cuda()
    a = hs.hsad_dwt(t, levels)
    gs, gl, gn = hs.hsad_dwest(a, c["inner"], c["outer"])
    torch.cuda.synchronize()
    idx = sample_pixels(512, 512, 400, seed=levels)
    ra = oracle.dwt_approx(s.cube, levels)
    rs, rl, rn = oracle.dwest(ra, c["inner"], c["outer"], idx=idx)
    e = score_rel_err(gs.cpu().numpy().ravel()[idx], rs)
    print("dwest 512x512x224 level", levels, err_summary(e), flush=True)
    assert e.max() <= TOL
    assert np.array_equal(gn.cpu().numpy().ravel()[idx], rn)


@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("levels,stats", [(5, 0), (4, 0), (4, 1), (3, 0)])
def test_dwest_tridiag_lane_groups(lanes, levels, stats):
    # 16, 32 or 64 lanes per pixel in the tridiagonalisation (4, 2 or 1 pixels per
    # wavefront) at L' = 7, 14 and 28; 13 x 11 = 143 pixels leave idle groups in the last
    # workgroup
    s = scene(500 + levels, 13, 11, 224)
    x = oracle.dwt_approx(s.cube, levels).astype(np.float32)
    L_ = hs.lib()
    try:
        assert L_.hsad_internal_dwest_lanes(lanes) == 0
        L_.hsad_internal_dwest_stats(stats)
        gs, gl, gn = _gpu(x, 3, 9)
    finally:
        L_.hsad_internal_dwest_lanes(0)
        L_.hsad_internal_dwest_stats(0)
    rs, rl, rn = oracle.dwest(x.astype(np.float64), 3, 9)
    assert np.array_equal(gn, rn)
    assert score_rel_err(gs, rs).max() <= TOL
    assert score_rel_err(gl, rl).max() <= TOL


def test_dwest_degenerate_and_short_spectra(solver):
    # L' = 1 and 2 (no reflection), a constant cube (C_diff = 0: no positive eigenvalue,
    # score 0) and a cube constant in one band
    for Lp in (1, 2, 3):
        x = np.random.default_rng(Lp).standard_normal((12, 13, Lp)).astype(np.float32)
        gs, gl, gn = _gpu(x, 3, 7)
        rs, rl, rn = oracle.dwest(x.astype(np.float64), 3, 7)
        assert np.array_equal(gn, rn)
        assert score_rel_err(gs, rs).max() <= TOL
    x = np.full((10, 11, 6), 0.25, dtype=np.float32)
    gs, gl, gn = _gpu(x, 3, 7)
    assert (gn == 0).all() and (gs == 0).all()
    x = np.random.default_rng(9).standard_normal((10, 11, 6)).astype(np.float32)
    x[..., 2] = 1.5
    gs, gl, gn = _gpu(x, 3, 7)
    rs, rl, rn = oracle.dwest(x.astype(np.float64), 3, 7)
    assert np.array_equal(gn, rn)
    assert score_rel_err(gs, rs).max() <= TOL


@pytest.mark.parametrize("stats", [1, 0])
@pytest.mark.parametrize("mode", [3, 0])
def test_dwest_runs_and_chunks_are_invariant(mode, stats):
    # A small workspace: with the Gram statistics it holds the QL columns of 8500 pixels and
    # the records of 8192, so a 100 x 100 image takes two runs (8500 + 1500 pixels), the first
    # in two Gram / tridiagonalisation chunks; with box statistics it holds one run of the
    # whole image and records of two bands of tile rows at a time.  Every pixel's arithmetic
    # is the same as with the default workspace, so the maps must equal the default's bit
    # for bit; sampled pixels of both runs are checked against the oracle.
    import torch
    H, W, Lp = 100, 100, 6
    x = np.random.default_rng(77).standard_normal((H, W, Lp)).astype(np.float32)
    x[..., 0] += np.linspace(0.0, 3.0, W, dtype=np.float32)[None, :]
    t = torch.from_numpy(x).cuda()
    L_ = hs.lib()
    L_.hsad_internal_dwest_solver(mode)
    L_.hsad_internal_dwest_stats(stats)
    try:
        s0, l0, n0 = hs.hsad_dwest(t, 3, 7)
        rec, col = (Lp + 2) * Lp * 8, 3 * Lp * 8
        ws = torch.empty(256 + rec * 8192 + col * 8500 + 100, dtype=torch.uint8, device="cuda")
        s1, l1, n1 = hs.hsad_dwest(t, 3, 7, ws=ws)
        torch.cuda.synchronize()
    finally:
        L_.hsad_internal_dwest_solver(0)
        L_.hsad_internal_dwest_stats(0)
    assert np.array_equal(s0.cpu().numpy(), s1.cpu().numpy())
    assert np.array_equal(l0.cpu().numpy(), l1.cpu().numpy())
    assert np.array_equal(n0.cpu().numpy(), n1.cpu().numpy())
    idx = np.array([0, 1, 99, 4321, 8191, 8192, 8499, 8500, 8501, 9998, 9999], dtype=np.int64)
    rs, rl, rn = oracle.dwest(x.astype(np.float64), 3, 7, idx=idx)
    assert np.array_equal(n1.cpu().numpy().ravel()[idx], rn)
    assert score_rel_err(s1.cpu().numpy().ravel()[idx], rs).max() <= TOL


def test_dwest_long_spectrum(solver):
    # L' = 100 (> 64: the QL kernel's LDS columns would hold only 16 pixels per workgroup,
    # so the default takes the run path); smooth spectra plus noise keep C_diff indefinite
    rng = np.random.default_rng(100)
    H, W, Lp = 11, 12, 100
    base = np.cumsum(rng.standard_normal((H, W, Lp)), axis=2) * 0.1
    x = (base + rng.standard_normal((H, W, Lp))).astype(np.float32)
    gs, gl, gn = _gpu(x, 3, 9)
    rs, rl, rn = oracle.dwest(x.astype(np.float64), 3, 9)
    print("dwest L'=100", solver, err_summary(score_rel_err(gs, rs)), flush=True)
    assert np.array_equal(gn, rn)
    assert score_rel_err(gs, rs).max() <= TOL
    assert score_rel_err(gl, rl).max() <= TOL


def test_dwest_full_band_paper_shape_sampled():
    # The paper's Img1 shape at full band (L' = 189) with 5 x 5 / 13 x 13 windows: the annulus
    # holds 144 samples, fewer than the bands, so C_outer is rank-deficient and C_diff has
    # many eigenvalues at rounding level.  Every pixel must converge (no NaN), and sampled
    # pixels must match the oracle.
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["img1_60x100x189"]
    sc = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"],
                          n_blob=c["n_blob"])
    t = torch.from_numpy(sc.cube).cuda()
    gs, gl, gn = hs.hsad_dwest(t, c["inner"], c["outer"])
    torch.cuda.synchronize()
    gs, gn = gs.cpu().numpy().ravel(), gn.cpu().numpy().ravel()
    assert np.isfinite(gs).all() and (gn >= 0).all()
    idx = sample_pixels(c["H"], c["W"], 40, seed=189)
    rs, rl, rn = oracle.dwest(sc.cube.astype(np.float64), c["inner"], c["outer"], idx=idx)
    e = score_rel_err(gs[idx], rs)
    print("img1 60x100x189 full band", err_summary(e), "npos mismatches", int((gn[idx] != rn).sum()), flush=True)
    assert np.array_equal(gn[idx], rn)
    assert e.max() <= TOL
