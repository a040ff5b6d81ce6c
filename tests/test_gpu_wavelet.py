"""GPU parity of the full transform [a_J d_J ... d_1] (Sec. 3, Fig. 1) and its inverse for
the Daubechies family (Haar to db16; Fig. 2 uses db16) against the FP64 oracle, plus
properties that hold at any size: perfect reconstruction, energy on even chains, and the
approximation band equal to hsad_dwt's.  Bound: per-pixel normwise relative error
<= 1e-5 (FP32 storage after FP64 arithmetic), as for the approximation-only DWT."""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from gpu_util import dwt_rel_err

pytestmark = pytest.mark.gpu


def _cube(seed, H, W, L):
    rng = np.random.default_rng(seed)
    base = rng.random(L).astype(np.float32)
    return (base + 0.1 * rng.standard_normal((H, W, L))).astype(np.float32)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [(224, 6), (189, 5), (64, 4), (7, 2), (256, 0), (33, 1), (430, 3), (2, 1), (3, 1)]


@pytest.mark.parametrize("order", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("L,levels", SHAPES)
def test_forward_and_inverse_match_oracle(order, L, levels):
    import torch
    print("wavelet case order=%d L=%d levels=%d" % (order, L, levels), flush=True)
    x = _cube(3000 + L + order, 9, 7, L)
    h = oracle.daubechies_lowpass(order)
    c = hs.hsad_dwt_full(_t(x), levels, order)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    ref = oracle.dwt_full_cube(x, levels, h)
    assert c.shape == ref.shape
    assert dwt_rel_err(c, ref) <= 1e-5
    # inverse on the same FP32 coefficients on both sides
    cf = ref.astype(np.float32)
    y = hs.hsad_idwt_full(_t(cf), L, levels, order)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    yref = oracle.idwt_full_cube(cf, L, levels, h)
    assert dwt_rel_err(y, yref) <= 1e-5
    # perfect reconstruction through the GPU pair
    z = hs.hsad_idwt_full(hs.hsad_dwt_full(_t(x), levels, order), L, levels, order)
    torch.cuda.synchronize()
    assert dwt_rel_err(z.cpu().numpy(), x.astype(np.float64)) <= 1e-5


@pytest.mark.parametrize("order", [1, 4, 16])
@pytest.mark.parametrize("L,levels", [(256, 4), (224, 5), (64, 6)])
def test_energy_on_even_chains(order, L, levels):
    import torch
    x = _cube(3100 + order, 6, 5, L)
    c = hs.hsad_dwt_full(_t(x), levels, order)
    torch.cuda.synchronize()
    c = c.cpu().numpy().astype(np.float64)
    ex = np.sum(x.astype(np.float64) ** 2, axis=-1)
    ec = np.sum(c ** 2, axis=-1)
    assert np.max(np.abs(ec - ex) / ex) <= 1e-6


@pytest.mark.parametrize("L,levels", [(224, 6), (224, 3), (189, 5), (430, 4)])
def test_approximation_band_equals_hsad_dwt(L, levels):
    import torch
    x = _cube(3200 + L, 17, 13, L)
    t = _t(x)
    c = hs.hsad_dwt_full(t, levels, 4)
    a = hs.hsad_dwt(t, levels)
    torch.cuda.synchronize()
    Lp = a.shape[-1]
    assert dwt_rel_err(c.cpu().numpy()[..., :Lp], a.cpu().numpy().astype(np.float64)) <= 1e-6


def test_constant_signal_has_no_detail():
    import torch
    x = np.full((4, 4, 256), 0.75, dtype=np.float32)
    for order in (1, 4, 16):
        c = hs.hsad_dwt_full(_t(x), 4, order)
        torch.cuda.synchronize()
        c = c.cpu().numpy().astype(np.float64)
        assert np.allclose(c[..., :16], 0.75 * 4.0, rtol=1e-6)
        assert np.max(np.abs(c[..., 16:])) <= 1e-6


def test_full_size_sampled():
    """512 x 512 x 224 cube, db4 and db16, J = 3: sampled pixels against the oracle, and the
    whole cube through the inverse."""
    import torch
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["cube_512x512x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
    t = torch.from_numpy(s.cube).cuda()
    rng = np.random.default_rng(7)
    idx = rng.choice(c["H"] * c["W"], 2000, replace=False)
    flat = s.cube.reshape(-1, c["L"])
    for order in (4, 16):
        print("wavelet full size order=%d" % order, flush=True)
        g = hs.hsad_dwt_full(t, 3, order)
        back = hs.hsad_idwt_full(g, c["L"], 3, order)
        torch.cuda.synchronize()
        gs = g.cpu().numpy().reshape(-1, g.shape[-1])[idx]
        ref = oracle.dwt_full_cube(flat[idx], 3, oracle.daubechies_lowpass(order))
        assert dwt_rel_err(gs, ref) <= 1e-5
        assert dwt_rel_err(back.cpu().numpy(), s.cube.astype(np.float64)) <= 1e-5
