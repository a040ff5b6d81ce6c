"""GPU parity of hsad_dwest (Sec. 2.2, eqs. 2-4) against the FP64 oracle.

Scores (||V_P^T m_diff||_2), literal scores (sum_P |v_i^T m_diff|) and the number of
positive eigenvalues are compared.  The score bound is an elementwise relative error
<= 1e-3, with a floor of 1e-3 * median.  The positive-eigenvalue counts must match
exactly.
"""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import err_summary, sample_pixels, scene, score_rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _gpu(x, inner, outer):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    s, lit, npos = hs.hsad_dwest(t, inner, outer)
    torch.cuda.synchronize()
    return s.cpu().numpy().ravel(), lit.cpu().numpy().ravel(), npos.cpu().numpy().ravel()


@pytest.mark.parametrize("H,W,levels,inner,outer", [
    (26, 21, 4, 3, 11), (17, 19, 3, 3, 11), (9, 10, 2, 3, 11), (20, 20, 6, 5, 13),
    (15, 33, 5, 1, 7), (6, 5, 4, 3, 5)])
def test_dwest_parity(H, W, levels, inner, outer):
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


@pytest.mark.parametrize("levels", [4, 3])
def test_dwest_full_size_sampled(levels):
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["C3"]
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
    print("C3 level", levels, err_summary(e), flush=True)
    assert e.max() <= TOL
    assert np.array_equal(gn.cpu().numpy().ravel()[idx], rn)
