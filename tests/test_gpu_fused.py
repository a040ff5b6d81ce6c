"""GPU tests of hsad_dwt_detect_fused: the DWT of one cube (Sec. 3) and the detection step
(LRX eq. 1, DWRX eq. 5, the eq. 12 threshold and its mask) on another, reduced cube, in one
launch where the two can share one; and of hsad_detect_stream_step, which also runs the eq. 12
threshold and mask of the cube before in the same launch.

Each workgroup of the shared launch runs the arithmetic of the kernel its role comes from,
so every output must equal that of hsad_dwt followed by hsad_detect bit for bit, for any
interleaving of the roles.  Where the pair cannot share a launch the call runs the two
kernels one after the other, with the same results.  The chain is also checked against the FP64 oracle: the reduced
cube to 1e-5 (as the DWT tests) and the scores to 1e-3 (as the detector tests).
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import dwt_rel_err, sample_pixels, scene, score_rel_err

pytestmark = pytest.mark.gpu


def _cube(seed, H, W, L):
    import torch
    return torch.from_numpy(scene(seed, H, W, L).cube).cuda()


def _np(t):
    return None if t is None else t.cpu().numpy()


def _same(a, b):
    if a is None or b is None:
        return a is None and b is None
    return np.array_equal(_np(a), _np(b), equal_nan=True)


def _set_run(run):
    assert hs.lib().hsad_internal_fused_run(int(run)) == 0


def _shares_launch(L, Lp, outer):
    """Whether hsad_dwt_detect_fused runs the pair as one launch: L' <= 5, L a multiple of 4
    and two workgroups' LDS (the larger of the 512-pixel DWT tile and the 32 x 16 detector
    tile with its default feature chunk) within 160 KiB."""
    if Lp > 5 or L % 4:
        return False
    R = outer // 2
    g = {1: 5, 2: 8, 3: 5, 4: 8, 5: 5}[Lp]
    ex, ey = 32 + 2 * R, 16 + 2 * R
    box = 16 * ex * (g | 1) * 8 + ey * ex * (Lp + 1) * 4
    return 2 * max(box, 512 * 33 * 4) <= 160 * 1024


# (H, W, L, levels, inner, outer).  L' = 4, 3, 2, 5, 1 share a launch; the last three run
# one after the other (L' = 6 > 5; L = 190 not a multiple of 4; a 21 x 21 window at L' = 4
# needs more LDS than two workgroups per CU allow).
CASES = [(512, 512, 224, 6, 5, 15), (37, 70, 64, 4, 3, 9), (33, 17, 96, 5, 1, 7),
         (20, 45, 128, 6, 0, 9), (61, 40, 160, 5, 3, 11), (16, 16, 32, 5, 1, 3), (9, 300, 224, 6, 5, 15),
         (30, 30, 192, 5, 3, 9), (30, 41, 190, 6, 3, 9), (40, 40, 64, 4, 3, 21)]


@pytest.mark.parametrize("H,W,L,levels,inner,outer", CASES)
@pytest.mark.parametrize("run", [128, 1, 7, 256])
def test_fused_equals_separate_calls(H, W, L, levels, inner, outer, run):
    import torch
    if run != 128 and H * W > 100000:
        pytest.skip("role interleaving is covered on the smaller images")
    print("fused", H, W, L, levels, inner, outer, "run", run, flush=True)
    nxt, cur = _cube(11 + H, H, W, L), _cube(12 + W, H, W, L)
    x = hs.hsad_dwt(cur, levels)
    Lp = x.shape[2]
    a_ref = hs.hsad_dwt(nxt, levels)
    l0, d0, s0, m0 = hs.hsad_detect(x, inner, outer, 1e-6, 3.0, dwrx=inner > 0)
    a = torch.full_like(a_ref, float("nan"))
    _set_run(run)
    try:
        l1, d1, s1, m1 = hs.hsad_dwt_detect_fused(nxt, levels, a, x, inner, outer, 1e-6, 3.0, dwrx=inner > 0)
        torch.cuda.synchronize()
    finally:
        _set_run(128)
    print("shares one launch:", _shares_launch(L, Lp, outer), flush=True)
    assert a.shape[2] == Lp
    assert _same(a, a_ref)
    assert _same(l1, l0) and _same(d1, d0) and _same(s1, s0) and _same(m1, m0)


def test_fused_against_oracle():
    import torch
    H, W, L, levels, inner, outer = 37, 70, 64, 4, 3, 9
    s_next, s_cur = scene(5, H, W, L), scene(6, H, W, L)
    x = torch.from_numpy(oracle.dwt_approx(s_cur.cube, levels).astype(np.float32)).cuda()
    a = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    lrx, dwrx, st, m = hs.hsad_dwt_detect_fused(torch.from_numpy(s_next.cube).cuda(), levels, a, x, inner, outer)
    torch.cuda.synchronize()
    assert dwt_rel_err(_np(a), oracle.dwt_approx(s_next.cube, levels)) <= 1e-5
    rl, rd = oracle.lrx_dwrx(_np(x).astype(np.float64), inner, outer, 1e-6)
    assert score_rel_err(_np(lrx), rl).max() <= 1e-3
    assert score_rel_err(_np(dwrx), rd).max() <= 1e-3
    tau = oracle.threshold(_np(lrx), 3.0)
    assert abs(_np(st)[3] - tau) <= 1e-12 * abs(tau)


def test_fused_full_size_sampled_against_oracle():
    # the headline shape and launch: 512 x 512 x 224, J = 6, windows 5 / 15; the oracle reduces
    # and scores a sample of pixels
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["cube_512x512x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"],
                         n_blob=c["n_blob"])
    t = torch.from_numpy(s.cube).cuda()
    x = hs.hsad_dwt(t, 6)
    a = torch.empty_like(x)
    lrx, dwrx, st, m = hs.hsad_dwt_detect_fused(t, 6, a, x, c["inner"], c["outer"], c["load_rel"])
    torch.cuda.synchronize()
    idx = sample_pixels(512, 512, 1500, seed=3)
    ra = oracle.dwt_approx(s.cube, 6)
    assert dwt_rel_err(_np(a).reshape(-1, 4)[idx], ra.reshape(-1, 4)[idx]) <= 1e-5
    rl, rd = oracle.lrx_dwrx(ra, c["inner"], c["outer"], c["load_rel"], idx=idx)
    assert score_rel_err(_np(lrx).ravel()[idx], rl).max() <= 1e-3
    assert score_rel_err(_np(dwrx).ravel()[idx], rd).max() <= 1e-3


def test_fused_pipeline_over_a_stream_of_cubes():
    # cube k is scored by the call that reduces cube k + 1; two reduced buffers alternate
    import torch
    H, W, L, levels, inner, outer = 48, 80, 224, 6, 5, 15
    cubes = [_cube(40 + k, H, W, L) for k in range(4)]
    bufs = [torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for _ in range(2)]
    got = []
    hs.hsad_dwt_detect_fused(cubes[0], levels, bufs[0], None, inner, outer)
    for k in range(len(cubes)):
        nxt = cubes[k + 1] if k + 1 < len(cubes) else None
        out = hs.hsad_dwt_detect_fused(nxt, levels, bufs[(k + 1) % 2] if nxt is not None else None, bufs[k % 2],
                                       inner, outer)
        got.append([t.clone() for t in out])
    torch.cuda.synchronize()
    for k, c in enumerate(cubes):
        ref = hs.hsad_detect(hs.hsad_dwt(c, levels), inner, outer)
        for g, r in zip(got[k], ref):
            assert _same(g, r), k


def test_fused_halves_alone():
    import torch
    H, W, L = 21, 34, 64
    c = _cube(7, H, W, L)
    a = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    assert hs.hsad_dwt_detect_fused(c, 4, a, None, 3, 9) == (None, None, None, None)
    assert _same(a, hs.hsad_dwt(c, 4))
    l1, d1, s1, m1 = hs.hsad_dwt_detect_fused(None, 4, None, a, 3, 9)
    l0, d0, s0, m0 = hs.hsad_detect(a, 3, 9)
    torch.cuda.synchronize()
    assert _same(l1, l0) and _same(d1, d0) and _same(s1, s0) and _same(m1, m0)


def test_fused_rejects_overlap_and_mismatch():
    import torch
    H, W, L = 16, 16, 64
    c = _cube(8, H, W, L)
    x = hs.hsad_dwt(c, 4)
    with pytest.raises(hs.HsadError) as e:
        hs.hsad_dwt_detect_fused(c, 4, x, x, 3, 9)               # writes the cube it scores
    assert e.value.code == hs.HSAD_EINVAL
    lrx = torch.empty(H * W * 4, dtype=torch.float32, device="cuda")
    with pytest.raises(hs.HsadError) as e:
        hs.hsad_dwt_detect_fused(c, 4, lrx.view(H, W, 4), x, 3, 9, lrx=lrx[: H * W].view(H, W))
    assert e.value.code == hs.HSAD_EINVAL
    big = torch.empty(H * W * L, dtype=torch.float32, device="cuda")
    big.copy_(c.reshape(-1))
    with pytest.raises(hs.HsadError) as e:                       # the detector would write the cube read
        hs.hsad_dwt_detect_fused(big.view(H, W, L), 4, torch.empty((H, W, 4), device="cuda"), x, 3, 9,
                                 lrx=big[: H * W].view(H, W))
    assert e.value.code == hs.HSAD_EINVAL
    with pytest.raises(hs.HsadError) as e:                       # L' 8 for the next cube, 4 for x
        hs.hsad_dwt_detect_fused(c, 3, torch.empty((H, W, 4), device="cuda"), x, 3, 9)
    assert e.value.code == hs.HSAD_EINVAL
    rc = hs.lib().hsad_dwt_detect_fused(None, 0, 0, None, None, H, W, 4, None, 3.0, None, None, None, None, None,
                                        0, None, None, None)
    assert rc == hs.HSAD_EINVAL
    torch.cuda.synchronize()


# hsad_detect_stream_step: the DWT of cube k + 1, the detector of cube k and the eq. (12)
# threshold + mask of cube k - 1 in one call (one launch where the first two can share one).
# 720 x 900 has more than 1024 tiles: its threshold stage runs after the shared launch.
STREAM = [(512, 512, 224, 6, 5, 15), (37, 70, 64, 4, 3, 9), (20, 45, 128, 6, 0, 9), (61, 40, 160, 5, 3, 11),
          (30, 41, 190, 6, 3, 9), (720, 900, 64, 4, 5, 15)]


@pytest.mark.parametrize("H,W,L,levels,inner,outer", STREAM)
@pytest.mark.parametrize("run", [128, 7])
def test_stream_step_equals_detect(H, W, L, levels, inner, outer, run):
    import torch
    if run != 128 and H * W > 100000:
        pytest.skip("role interleaving is covered on the smaller images")
    print("stream", H, W, L, levels, inner, outer, "run", run, flush=True)
    cubes = [_cube(60 + k + H, H, W, L) for k in range(3)]
    Lp = hs.hsad_dwt_out_len(L, levels)
    A = [torch.empty((H, W, Lp), dtype=torch.float32, device="cuda") for _ in range(2)]
    S = [torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(2)]
    nws = hs.hsad_detect_workspace_bytes(H, W, Lp, inner, outer, 1e-6)
    WS = [torch.empty(nws, dtype=torch.uint8, device="cuda") for _ in range(2)]
    dw = torch.empty((H, W), dtype=torch.float32, device="cuda") if inner > 0 else None
    got = [dict() for _ in cubes]
    _set_run(run)
    try:
        hs.hsad_detect_stream_step(cubes[0], levels, A[0], None, inner, outer, None, None, H=H, W=W, Lp=Lp)
        for k in range(len(cubes) + 1):
            nxt = cubes[k + 1] if k + 1 < len(cubes) else None
            x = A[k % 2] if k < len(cubes) else None
            st = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
            mk = torch.full((H, W), 7, dtype=torch.uint8, device="cuda")
            hs.hsad_detect_stream_step(nxt, levels, A[(k + 1) % 2] if nxt is not None else None, x, inner, outer,
                                       S[k % 2] if x is not None else None, WS[k % 2] if x is not None else None,
                                       dwrx=dw if x is not None else None,
                                       prev_lrx=S[(k - 1) % 2] if k >= 1 else None,
                                       prev_ws=WS[(k - 1) % 2] if k >= 1 else None,
                                       prev_stats=st if k >= 1 else None, prev_mask=mk if k >= 1 else None,
                                       H=H, W=W, Lp=Lp)
            if x is not None:
                got[k]["lrx"] = S[k % 2].clone()
                got[k]["dwrx"] = dw.clone() if dw is not None else None
            if k >= 1:
                got[k - 1]["stats"], got[k - 1]["mask"] = st, mk
        torch.cuda.synchronize()
    finally:
        _set_run(128)
    for k, c in enumerate(cubes):
        l0, d0, s0, m0 = hs.hsad_detect(hs.hsad_dwt(c, levels), inner, outer, 1e-6, 3.0, dwrx=inner > 0)
        torch.cuda.synchronize()
        assert _same(got[k]["lrx"], l0) and _same(got[k]["dwrx"], d0), k
        assert _same(got[k]["stats"], s0) and _same(got[k]["mask"], m0), k


def test_stream_step_rejects_bad_arguments():
    import torch
    H, W, L = 16, 16, 64
    c = _cube(9, H, W, L)
    x = hs.hsad_dwt(c, 4)
    lrx = torch.empty((H, W), device="cuda")
    ws = torch.empty(hs.hsad_detect_workspace_bytes(H, W, 4, 3, 9, 1e-6), dtype=torch.uint8, device="cuda")
    st = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(hs.HsadError) as e:                       # nothing to do
        hs.hsad_detect_stream_step(None, 4, None, None, 3, 9, None, None, H=H, W=W, Lp=4)
    assert e.value.code == hs.HSAD_EINVAL
    with pytest.raises(hs.HsadError) as e:                       # the threshold reads the partials being written
        hs.hsad_detect_stream_step(None, 4, None, x, 3, 9, lrx, ws, prev_lrx=lrx.clone(), prev_ws=ws, prev_stats=st)
    assert e.value.code == hs.HSAD_EINVAL
    with pytest.raises(hs.HsadError) as e:                       # L' 14: not the box path's sizes for the stream
        hs.hsad_detect_stream_step(None, 2, None, hs.hsad_dwt(_cube(10, H, W, 56), 2), 3, 9, lrx,
                                   torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.code == hs.HSAD_EUNSUPPORTED
    torch.cuda.synchronize()
