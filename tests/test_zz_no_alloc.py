"""hsad_detect_noalloc (workspace from the library's static device scratch) against
hsad_detect (caller workspace): the same kernels, so every output must agree bitwise, on
two calls in a row where the second has a smaller image (the scratch keeps the first
call's contents).  Also checked against the FP64 oracle at the LRX bound.  Three paths:
box sums (L' = 4), box statistics + Cholesky (L' = 14) and the matrix-core Gram (L' = 14
with a 33 x 33 window)."""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import scene, score_rel_err

pytestmark = pytest.mark.gpu


def _reduced(seed, H, W, levels):
    s = scene(seed, H, W, 224)
    return oracle.dwt_approx(s.cube, levels).astype(np.float32)


def _both(x, inner, outer):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ref = hs.hsad_detect(t, inner, outer, 1e-6, 3.0)
    got = hs.hsad_detect_noalloc(t, inner, outer, 1e-6, 3.0)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in ref], [a.cpu().numpy() for a in got]


@pytest.mark.parametrize("levels,inner,outer", [(6, 5, 15), (4, 5, 15), (4, 3, 33)])
def test_noalloc_matches_detect_twice(levels, inner, outer):
    for call, (H, W) in enumerate(((72, 88), (40, 26))):
        print("noalloc case levels=%d inner=%d outer=%d call=%d shape=%dx%d" % (levels, inner, outer, call, H, W),
              flush=True)
        x = _reduced(1700 + call, H, W, levels)
        ref, got = _both(x, inner, outer)
        for a, b, name in zip(ref, got, ("lrx", "dwrx", "stats", "mask")):
            assert a.shape == b.shape, name
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), name
        rl, rd = oracle.lrx_dwrx(x.astype(np.float64), inner, outer, 1e-6)
        assert score_rel_err(got[0], rl).max() <= 1e-3
        assert score_rel_err(got[1], rd).max() <= 1e-3
        tau = oracle.threshold(rl, 3.0)
        assert abs(float(got[2][3]) - tau) <= 1e-3 * abs(tau)
