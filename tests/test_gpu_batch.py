"""GPU parity of the persistent batch engine (uneven scenes in one plan).

Every scene of the batch must agree with the FP64 oracle chain within the same bounds
as the single-scene calls (DWT + LRX/DWRX, 1e-3 relative with a floor of 1e-3 * median).
A replayed HIP graph must reproduce the eager run bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import err_summary, scene, score_rel_err

pytestmark = pytest.mark.gpu


def _specs():
    # a small uneven batch: the fused box bucket (L' <= 8), the box-statistics bucket
    # (L' <= 64, outer <= 31) and the Gram bucket; odd L, ragged sizes
    return [
        dict(seed=1, H=37, W=29, L=224, levels=6, inner=5, outer=15),    # L' = 4 (box)
        dict(seed=2, H=20, W=41, L=189, levels=5, inner=3, outer=13),    # L' = 6 (box)
        dict(seed=3, H=19, W=23, L=131, levels=3, inner=3, outer=9),     # L' = 17 (box statistics)
        dict(seed=4, H=24, W=17, L=224, levels=4, inner=5, outer=11),    # L' = 14 (box statistics)
        dict(seed=5, H=9, W=33, L=430, levels=2, inner=7, outer=21),     # L' = 108 (gram)
        dict(seed=6, H=31, W=16, L=100, levels=5, inner=1, outer=9),     # L' = 4 (box)
        dict(seed=7, H=22, W=19, L=160, levels=3, inner=3, outer=33),    # L' = 20, outer 33 (gram)
    ]


def _build(specs, options=None):
    import torch
    scs, cubes = [], []
    for sp in specs:
        s = scene(sp["seed"], sp["H"], sp["W"], sp["L"])
        cubes.append(s)
        scs.append(dict(cube=torch.from_numpy(s.cube).cuda(), levels=sp["levels"], inner=sp["inner"],
                        outer=sp["outer"], load_rel=1e-6))
    return hs.BatchPlan(scs, options), cubes


def test_batch_matches_oracle():
    import torch
    specs = _specs()
    plan, scenes = _build(specs)
    print(plan.info())
    plan.run()
    torch.cuda.synchronize()
    for sp, s, gl, gd in zip(specs, scenes, plan.lrx, plan.dwrx):
        ra = oracle.dwt_approx(s.cube, sp["levels"])
        rl, rd = oracle.lrx_dwrx(ra, sp["inner"], sp["outer"], 1e-6)
        el = score_rel_err(gl.cpu().numpy().ravel(), rl)
        ed = score_rel_err(gd.cpu().numpy().ravel(), rd)
        print(sp, "lrx", err_summary(el), "dwrx", err_summary(ed), flush=True)
        assert el.max() <= 1e-3 and ed.max() <= 1e-3
    plan.close()


def test_batch_graph_replay_and_options():
    import torch
    opt = hs.batch_default_options()
    opt.wgs_per_cu = 1
    opt.chunk_bytes = 2 << 20          # forces several Gram chunks
    opt.dwt_pixels = 5
    plan, scenes = _build(_specs(), opt)
    assert plan.info()["gram_chunks"] > 1
    plan.run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in plan.lrx] + [t.clone() for t in plan.dwrx]
    for t in plan.lrx + plan.dwrx:
        t.fill_(-1.0)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run(stream=s)
    for rep in range(3):
        for t in plan.lrx + plan.dwrx:
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in plan.lrx] + [t.clone() for t in plan.dwrx]
        for a, b in zip(eager, got):
            assert torch.equal(a, b), "graph replay %d differs" % rep
    plan.close()


def test_batch_rejects_bad_scenes():
    import torch
    c = torch.zeros((8, 8, 64), device="cuda")
    with pytest.raises(hs.HsadError):
        hs.BatchPlan([dict(cube=c, levels=2, inner=4, outer=9)])
    with pytest.raises(hs.HsadError):      # L' = 150 > 128
        hs.BatchPlan([dict(cube=torch.zeros((8, 8, 300), device="cuda"), levels=1, inner=3, outer=9)])
