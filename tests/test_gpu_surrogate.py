"""GPU checks of the learned LRX surrogate against the FP64 oracle (oracle/mlp.py).

Bounds:
  features (FP64 sums, FP32 output)   rtol 1e-5, atol 1e-6
  packing and the BF16 weight copy    bitwise (same FP32 operations, round to nearest even)
  network forward / gradient          normwise relative 2e-2 / 1e-2 per parameter block:
                                      the kernels round the hidden activations and the
                                      back-propagated errors to BF16 (unit roundoff 2^-9)
                                      before each product and accumulate in FP32; the
                                      oracle is FP64 on the same BF16 weights and inputs.
                                      The ReLU derivative jumps at zero, so for the
                                      gradient both sides take the sign decisions in the
                                      kernels' precision (BF16 operands, FP32 sums)
  Adam step on a given gradient       each stage (moments, update) against FP64 applied to
                                      the GPU's inputs of that stage, within 2^-21 times
                                      the operand magnitudes (a few FP32 units)
  selection flags and counts          bitwise (SplitMix64 on both sides, same FP64 test)
  exact LRX at listed pixels          1e-3 relative vs the oracle; bitwise vs the full map
                                      through the same statistics (matrix-core Gram) and
                                      Cholesky kernels
  hybrid map                          exact LRX on the selected pixels (bitwise),
                                      expm1(prediction) elsewhere, eq. (12) mask
The trained network's accuracy itself has no exact counterpart ("parity unpinned"): it is
judged by the audit against exact LRX and by the change of ROC AUC.
"""
import numpy as np
import pytest

import oracle
import paper_1201_2025_amd as hs
from oracle import mlp
from gpu_util import sample_pixels, scene, score_rel_err, err_summary

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def _reduced(seed, H, W, Lp, L=224, n_single=None):
    """FP32 reduced cube from the oracle's DWT of a generated scene; when no level of L
    bands gives L', a generated scene of L' bands stands in for it."""
    lv = [j for j in range(12) if oracle.dwt_out_len(L, j) == Lp]
    if not lv:
        s = scene(seed, H, W, Lp, n_single=n_single)
        return s.cube, s
    s = scene(seed, H, W, L, n_single=n_single)
    return oracle.dwt_approx(s.cube, lv[0]).astype(np.float32), s


def _bf16_round(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def _bf16_bits(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).view(torch.int16).numpy()


def _bits_to_f32(bits):
    b = np.asarray(bits, dtype=np.int16).astype(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


# ---------------------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------------------
FEAT = [(37, 29, 14, 5, 15), (20, 23, 5, 0, 9), (16, 40, 2, 1, 13), (45, 50, 7, 3, 45),
        (70, 66, 3, 5, 63), (1, 1, 4, 0, 3), (3, 2, 14, 1, 3), (33, 31, 56, 3, 11)]


# tile width: 32 where its LDS fits (the default) or 16, through the library's internal switch
@pytest.mark.parametrize("tile", ["default", "w16"])
@pytest.mark.parametrize("H,W,Lp,inner,outer", FEAT)
def test_features_parity(H, W, Lp, inner, outer, tile):
    print("features", H, W, Lp, inner, outer, tile, flush=True)
    import torch
    x, _ = _reduced(300 + Lp, H, W, Lp)
    L_ = hs.lib()
    L_.hsad_internal_feat_cfg(1 if tile == "w16" else 0)
    try:
        f = hs.hsad_surrogate_features(_t(x), inner, outer)
        torch.cuda.synchronize()
    finally:
        L_.hsad_internal_feat_cfg(0)
    got = f.cpu().numpy()
    idx = sample_pixels(H, W, 400, seed=Lp)
    ref = mlp.features(x.astype(np.float64), inner, outer, idx)
    assert got.shape == (H * W, 3 * Lp)
    assert np.allclose(got[idx], ref, rtol=1e-5, atol=1e-6), np.abs(got[idx] - ref).max()


def test_norm_stats_and_packing():
    import torch
    x, _ = _reduced(311, 41, 37, 14)
    xt = _t(x)
    f = hs.hsad_surrogate_features(xt, 5, 15)
    norm = hs.hsad_mlp_norm_stats(f)
    D, Dp, _, _ = hs.hsad_mlp_dims(14)
    X = hs.hsad_mlp_pack(f, norm, Dp)
    Xd = hs.hsad_surrogate_features(xt, 5, 15, norm=norm, Dp=Dp)
    torch.cuda.synchronize()
    fn = f.cpu().numpy().astype(np.float64)
    nm = norm.cpu().numpy()
    assert np.allclose(nm[0::2], fn.mean(0), rtol=1e-6, atol=1e-7)
    assert np.allclose(1.0 / nm[1::2], fn.std(0), rtol=1e-5)
    # same FP32 operations -> same BF16 bits
    fs = f.cpu().numpy()
    ref = _bf16_bits((fs - nm[0::2]) * nm[1::2])
    Xc = X.cpu().numpy()
    assert np.array_equal(Xc[:, :D], ref)
    assert np.all(Xc[:, D:] == 0)
    assert np.array_equal(Xd.cpu().numpy(), Xc)


# ---------------------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------------------
def _rand_params(seed, Dp, D=None):
    r = np.random.default_rng(seed)
    D = Dp if D is None else D
    W1 = np.zeros((Dp, 128))
    W1[:D] = r.standard_normal((D, 128)) * np.sqrt(2.0 / D)
    b1 = r.standard_normal(128) * 0.1
    W2 = r.standard_normal((128, 128)) * np.sqrt(2.0 / 128)
    b2 = r.standard_normal(128) * 0.1
    w3 = r.standard_normal(128) * np.sqrt(1.0 / 128)
    return mlp.pack(W1, b1, W2, b2, w3, 0.05).astype(np.float32)


def _as_kernel_sees(p, Dp):
    """FP64 parameters with W1 and W2 rounded to BF16 (the matrix-core operands)."""
    q = p.astype(np.float64).copy()
    nW1 = Dp * 128
    q[:nW1] = _bf16_round(p[:nW1])
    o = nW1 + 128
    q[o:o + 128 * 128] = _bf16_round(p[o:o + 128 * 128])
    return q


def _model(p, Dp):
    import torch
    P = _t(p)
    wbf = torch.empty(128 * Dp + 2 * 128 * 128, dtype=torch.int16, device="cuda")
    hs.hsad_mlp_sync(P, Dp, wbf)
    return P, wbf


@pytest.mark.parametrize("Dp", [32, 64, 192, 256])
def test_sync_layout(Dp):
    import torch
    p = _rand_params(1 + Dp, Dp)
    P, wbf = _model(p, Dp)
    torch.cuda.synchronize()
    w = wbf.cpu().numpy()
    W1, _, W2, _, _, _ = mlp.unpack(p, Dp)
    n1 = 128 * Dp
    assert np.array_equal(w[:n1].reshape(128, Dp), _bf16_bits(W1.T.astype(np.float32)))
    assert np.array_equal(w[n1:n1 + 16384].reshape(128, 128), _bf16_bits(W2.T.astype(np.float32)))
    assert np.array_equal(w[n1 + 16384:].reshape(128, 128), _bf16_bits(W2.astype(np.float32)))


@pytest.mark.parametrize("Dp,n", [(32, 1), (64, 15), (64, 17), (192, 1000), (256, 4099), (64, 70001)])
def test_infer_parity(Dp, n):
    print("infer", Dp, n, flush=True)
    import torch
    r = np.random.default_rng(Dp + n)
    p = _rand_params(Dp, Dp)
    Xf = _bf16_round(r.standard_normal((n, Dp)))
    X = _t(_bf16_bits(Xf))
    P, wbf = _model(p, Dp)
    y = hs.hsad_mlp_infer(X, P, wbf)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    ref = mlp.forward(Xf.astype(np.float64), _as_kernel_sees(p, Dp), Dp)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("infer normwise", err, flush=True)
    assert err <= 2e-2
    assert np.all(np.isfinite(got))


def _kernel_masks(Xf, p, Dp):
    """ReLU decisions taken in the kernels' precision: BF16 operands, FP32 sums, h1 rounded
    to BF16 before the second product."""
    W1, b1, W2, b2, _, _ = mlp.unpack(p, Dp)
    X32 = np.asarray(Xf, dtype=np.float32)
    a1 = X32 @ _bf16_round(W1.astype(np.float32)) + b1.astype(np.float32)
    h1 = _bf16_round(np.maximum(a1, 0))
    a2 = h1 @ _bf16_round(W2.astype(np.float32)) + b2.astype(np.float32)
    return a1 > 0, a2 > 0


def _blocks(g, Dp):
    W1, b1, W2, b2, w3, b3 = mlp.unpack(g, Dp)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "w3": w3, "b3": np.array([b3])}


@pytest.mark.parametrize("Dp,batch,nrows", [(64, 64, 500), (64, 1000, 3000), (192, 777, 2000), (32, 5, 9)])
def test_gradient_parity(Dp, batch, nrows):
    print("gradient", Dp, batch, nrows, flush=True)
    import torch
    r = np.random.default_rng(7 * Dp + batch)
    p = _rand_params(Dp + 3, Dp)
    Xf = _bf16_round(r.standard_normal((nrows, Dp)))
    tgt = (r.standard_normal(nrows) + 1.0).astype(np.float32)
    tgt[r.choice(nrows, max(1, nrows // 50), replace=False)] = np.nan
    rows = r.choice(nrows, batch, replace=False).astype(np.int32)
    P, wbf = _model(p, Dp)
    g = hs.hsad_mlp_gradient(_t(_bf16_bits(Xf)), _t(tgt), _t(rows), P, wbf)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    loss, gr = mlp.loss_and_grad(Xf[rows].astype(np.float64), tgt[rows].astype(np.float64),
                                 _as_kernel_sees(p, Dp), Dp, masks=_kernel_masks(Xf[rows], p, Dp))
    assert abs(g[-1] - loss) <= 1e-2 * loss
    gb, rb = _blocks(g[:-1], Dp), _blocks(gr, Dp)
    for k in gb:
        e = np.linalg.norm(gb[k] - rb[k]) / max(np.linalg.norm(rb[k]), 1e-30)
        print("grad block", k, e, flush=True)
        assert e <= 1e-2, k
    assert np.all(g[-4:-1] == 0)


def test_train_step_is_gradient_plus_adam():
    import torch
    Dp, nrows, batch = 64, 4000, 1500
    r = np.random.default_rng(99)
    p = _rand_params(5, Dp, D=42)
    X = _t(_bf16_bits(_bf16_round(r.standard_normal((nrows, Dp)))))
    tgt = _t((r.standard_normal(nrows) + 2.0).astype(np.float32))
    rows = _t(r.choice(nrows, batch, replace=False).astype(np.int32))
    npar = p.size
    m0 = (r.standard_normal(npar) * 1e-3).astype(np.float32)
    v0 = (np.abs(r.standard_normal(npar)) * 1e-5).astype(np.float32)
    for step, lr in [(1, 1e-3), (7, 3e-3)]:
        P, wbf = _model(p, Dp)
        g = hs.hsad_mlp_gradient(X, tgt, rows, P, wbf)
        m_in = m0 if step > 1 else np.zeros_like(m0)
        v_in = v0 if step > 1 else np.zeros_like(v0)
        M, V = _t(m_in), _t(v_in)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        hs.hsad_mlp_train_step(X, tgt, rows, P, wbf, M, V, step, lr, loss=loss)
        torch.cuda.synchronize()
        gn = g.cpu().numpy().astype(np.float64)
        assert loss.item() == g[-1].item()
        g64 = gn[:-1]
        # each stage against FP64 applied to the GPU's inputs of that stage; FP32 arithmetic
        # and stores allow a few units in the last place of the operands (2^-21 relative)
        _, me, ve = mlp.adam_step(p.astype(np.float64), g64, m_in, v_in, step, lr)
        Mg, Vg = M.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(Mg - me) <= 2.0 ** -21 * (0.9 * np.abs(m_in) + 0.1 * np.abs(g64)) + 1e-30)
        assert np.all(np.abs(Vg - ve) <= 2.0 ** -21 * (0.999 * v_in + 0.001 * g64 * g64) + 1e-30)
        upd = lr * (Mg / (1 - 0.9 ** step)) / (np.sqrt(Vg / (1 - 0.999 ** step)) + 1e-8)
        pe = p.astype(np.float64) - upd
        Pg = P.cpu().numpy()
        bad = np.abs(Pg - pe) > 2.0 ** -21 * (np.abs(p) + np.abs(upd)) + 1e-30
        if bad.any():
            k = np.nonzero(bad)[0][:8]
            print("adam mismatch", step, bad.sum(), k, gn[k], p[k], Pg[k], pe[k], flush=True)
        assert not bad.any()
        # the BF16 copy follows the updated weights bitwise
        Pn = P.cpu().numpy()
        W1, _, W2, _, _, _ = mlp.unpack(Pn, Dp)
        w = wbf.cpu().numpy()
        assert np.array_equal(w[:128 * Dp].reshape(128, Dp), _bf16_bits(W1.T.astype(np.float32)))
        assert np.array_equal(w[128 * Dp + 16384:].reshape(128, 128), _bf16_bits(W2.astype(np.float32)))


def test_gradient_deterministic():
    import torch
    Dp = 64
    r = np.random.default_rng(3)
    p = _rand_params(11, Dp)
    X = _t(_bf16_bits(_bf16_round(r.standard_normal((5000, Dp)))))
    tgt = _t(r.standard_normal(5000).astype(np.float32))
    rows = _t(r.permutation(5000).astype(np.int32))
    P, wbf = _model(p, Dp)
    a = hs.hsad_mlp_gradient(X, tgt, rows, P, wbf).cpu().numpy()
    b = hs.hsad_mlp_gradient(X, tgt, rows, P, wbf).cpu().numpy()
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------------------
# selection, error statistics, exact LRX at listed pixels
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 63, 65, 1000003])
def test_select_parity(n):
    print("select", n, flush=True)
    import torch
    r = np.random.default_rng(n)
    y = (r.standard_normal(n) * 2 + 3).astype(np.float32)
    if n > 5:
        y[3] = np.nan
    tau = 20.0
    stats = _t(np.array([n, 0.0, 1.0, tau]))
    seed, frac, band = 0xDEADBEEF12345678, 0.01, 0.3
    flags, idx, counts = hs.hsad_surrogate_select(_t(y), stats, band, seed, frac)
    torch.cuda.synchronize()
    ref = mlp.select(y, tau, band, seed, frac)
    f = flags.cpu().numpy()
    assert np.array_equal(f, ref)
    c = counts.cpu().numpy()
    assert c[0] == (ref > 0).sum() and c[1] == (ref & 1).sum() and c[2] == ((ref & 2) > 0).sum()
    sel = idx.cpu().numpy()[:c[0]]
    assert np.array_equal(sel, np.nonzero(ref)[0])      # ascending, deterministic


def test_error_stats():
    import torch
    r = np.random.default_rng(5)
    n = 300001
    y = r.standard_normal(n).astype(np.float32)
    s = np.abs(r.standard_normal(n) * 5).astype(np.float32)
    s[7] = np.inf
    flags = r.integers(0, 4, n).astype(np.uint8)
    out = hs.hsad_error_stats(_t(y), _t(s), True, _t(flags), 2)
    torch.cuda.synchronize()
    sel = (flags & 2) > 0
    e = y[sel].astype(np.float64) - np.log1p(s[sel].astype(np.float64))
    e = e[np.isfinite(e)]
    o = out.cpu().numpy()
    assert o[0] == e.size
    assert np.isclose(o[1], np.sqrt(np.mean(e * e)), rtol=1e-12)
    assert np.isclose(o[2], np.abs(e).max(), rtol=1e-15)
    o2 = hs.hsad_error_stats(_t(y), _t(np.log1p(s)), False).cpu().numpy()
    ok = np.isfinite(np.log1p(s))
    e2 = y[ok].astype(np.float64) - np.log1p(s[ok]).astype(np.float32).astype(np.float64)
    assert o2[0] == ok.sum() and np.isclose(o2[1], np.sqrt(np.mean(e2 * e2)), rtol=1e-12)


@pytest.mark.parametrize("H,W,Lp,inner,outer", [(37, 29, 14, 5, 15), (30, 31, 6, 3, 9), (25, 20, 28, 1, 13)])
def test_lrx_dwrx_at(H, W, Lp, inner, outer):
    print("lrx at", H, W, Lp, inner, outer, flush=True)
    import torch
    x, _ = _reduced(400 + Lp, H, W, Lp)
    xt = _t(x)
    r = np.random.default_rng(Lp)
    idx = np.concatenate([sample_pixels(H, W, 200, seed=Lp), r.integers(0, H * W, 20)]).astype(np.int32)
    lrx = torch.full((H, W), -1.0, device="cuda")
    dwrx = torch.full((H, W), -1.0, device="cuda")
    hs.hsad_lrx_dwrx_at(xt, _t(idx), inner, outer, 1e-6, lrx=lrx, dwrx=dwrx)
    # tiny workspace: one pixel per chunk
    lrx1 = torch.full((H, W), -1.0, device="cuda")
    hs.hsad_lrx_dwrx_at(xt, _t(idx[:40]), inner, outer, 1e-6, lrx=lrx1, ws_bytes=(Lp + 2) * Lp * 8)
    L_ = hs.lib()
    try:       # the full maps through the same statistics (matrix-core Gram) and Cholesky
        L_.hsad_internal_generic_force(1)
        fl, fd = hs.hsad_lrx_dwrx(xt, inner, outer, 1e-6)
    finally:
        L_.hsad_internal_generic_force(-1)
    torch.cuda.synchronize()
    gl, gd = lrx.cpu().numpy().ravel(), dwrx.cpu().numpy().ravel()
    untouched = np.ones(H * W, bool)
    untouched[idx] = False
    assert np.all(gl[untouched] == -1) and np.all(gd[untouched] == -1)
    u = np.unique(idx)
    rl, rd = oracle.lrx_dwrx(x.astype(np.float64), inner, outer, 1e-6, idx=u)
    el, ed = score_rel_err(gl[u], rl), score_rel_err(gd[u], rd)
    print("lrx_at", err_summary(el), "dwrx_at", err_summary(ed), flush=True)
    assert el.max() <= 1e-3 and ed.max() <= 1e-3
    assert np.array_equal(lrx1.cpu().numpy().ravel()[idx[:40]], gl[idx[:40]])
    if Lp > 8:
        assert np.array_equal(gl[u], fl.cpu().numpy().ravel()[u])
        assert np.array_equal(gd[u], fd.cpu().numpy().ravel()[u])


# ---------------------------------------------------------------------------------------
# training and the hybrid map
# ---------------------------------------------------------------------------------------
LV, LP, IN, OUT = 4, 14, 5, 15


def _train(seed=0, n_scenes=10, size=96, epochs=12):
    import torch
    sur = hs.Surrogate(LP, IN, OUT, 1e-6, seed=seed)
    for i in range(n_scenes):
        s = scene(2000 + i, size, size, 224, K=6, n_single=size * size // 600, n_blob=2)
        sur.add_scene(_t(s.cube), LV)
    hist = sur.fit(epochs=epochs, batch=2048, lr=3e-3, lr_final=2e-4, val_scenes=2, seed=seed)
    torch.cuda.synchronize()
    return sur, hist


@pytest.fixture(scope="module")
def trained():
    return _train()


def test_training_learns(trained):
    sur, hist = trained
    print("history", hist, flush=True)
    assert hist[-1][0] < 0.6 * hist[0][0]
    # better than the best constant on the held-out scenes (whose targets are the last rows)
    t = sur.tgt_train.cpu().numpy()[-2 * 96 * 96:].astype(np.float64)
    const = np.sqrt(np.mean((t - t.mean()) ** 2))
    print("validation rmse %.4f, best constant %.4f" % (sur.rmse_val, const), flush=True)
    assert sur.rmse_val < const
    assert sur.rmse_val == min(h[1] for h in hist)


def test_training_deterministic(trained):
    sur, _ = trained
    again, _ = _train()
    assert np.array_equal(sur.params.cpu().numpy(), again.params.cpu().numpy())


def _hybrid_case(sur, seed=2100, size=160, gram=False):
    import torch
    s = scene(seed, size, size, 224, K=6, n_single=size * size // 600, n_blob=4)
    x = hs.hsad_dwt(_t(s.cube), LV)
    L_ = hs.lib()
    try:
        L_.hsad_internal_generic_force(1 if gram else -1)
        exact = hs.hsad_lrx(x, IN, OUT)
    finally:
        L_.hsad_internal_generic_force(-1)
    yhat = sur.predict(x)
    torch.cuda.synchronize()
    return s, x, exact, yhat


def test_hybrid_map(trained):
    import torch
    sur, _ = trained
    s, x, exact, yhat = _hybrid_case(sur, gram=True)      # the recompute's own statistics path
    exact_auto = hs.hsad_lrx(x, IN, OUT).cpu().numpy().ravel()
    seed, frac, band_k, z = 77, 0.01, 3.0, 3.0
    scores, mask, rep = sur.run(x, z_alpha=z, band_k=band_k, audit_frac=frac, fallback_factor=4.0, seed=seed)
    torch.cuda.synchronize()
    print("report", rep, flush=True)
    y = yhat.cpu().numpy().ravel()
    sc, ex = scores.cpu().numpy().ravel(), exact.cpu().numpy().ravel()
    # eq. (12) on the predicted scores
    pred = np.expm1(y.astype(np.float64)).astype(np.float32)
    tau_p = oracle.threshold(pred.astype(np.float64), z)
    assert np.isclose(rep["tau_pred"], tau_p, rtol=1e-6)
    flags = mlp.select(y, rep["tau_pred"], band_k * sur.rmse_val, seed, frac)
    assert rep["fallback"] == 0
    assert rep["selected"] == (flags > 0).sum() and rep["band"] == (flags & 1).sum()
    assert rep["audit"] == ((flags & 2) > 0).sum()
    sel = flags > 0
    assert np.array_equal(sc[sel], ex[sel])
    assert score_rel_err(sc[sel], exact_auto[sel]).max() <= 1e-3     # and the default exact map
    assert np.allclose(sc[~sel], pred[~sel], rtol=1e-6)
    ea = y[(flags & 2) > 0].astype(np.float64) - np.log1p(ex[(flags & 2) > 0].astype(np.float64))
    assert np.isclose(rep["audit_rmse"], np.sqrt(np.mean(ea * ea)), rtol=1e-9)
    tau_f = oracle.threshold(sc.astype(np.float64), z)
    assert np.isclose(rep["tau"], tau_f, rtol=1e-9)
    assert np.array_equal(mask.cpu().numpy().ravel(), (sc > rep["tau"]).astype(np.uint8))
    # what the surrogate does to detection quality: AUC of the hybrid map vs exact LRX
    a_h = oracle.auc(sc.astype(np.float64), s.truth.ravel())
    a_e = oracle.auc(ex.astype(np.float64), s.truth.ravel())
    print("AUC exact %.6f hybrid %.6f delta %.2e selected %.3f" % (a_e, a_h, a_h - a_e, rep["selected"] / sc.size),
          flush=True)
    assert abs(a_h - a_e) <= 2e-3


def test_hybrid_fallback_on_poisoned_weights(trained):
    import torch
    sur, _ = trained
    _, x, exact, _ = _hybrid_case(sur, seed=2101, size=64)
    bad = hs.Surrogate(LP, IN, OUT, 1e-6)
    bad.params.copy_(sur.params)
    off_b3 = sur.Dp * 128 + 3 * 128 + 128 * 128
    bad.params[off_b3] += 5.0          # predictions shifted by 5 in log1p space
    hs.hsad_mlp_sync(bad.params, bad.Dp, bad.wbf)
    bad.norm, bad.rmse_val = sur.norm, sur.rmse_val
    scores, mask, rep = bad.run(x, band_k=3.0, audit_frac=0.05, fallback_factor=2.0, seed=1)
    torch.cuda.synchronize()
    assert rep["fallback"] == 1 and rep["selected"] == x.shape[0] * x.shape[1]
    assert rep["audit_rmse"] > 2.0 * sur.rmse_val
    assert np.array_equal(scores.cpu().numpy(), exact.cpu().numpy())


def test_checkpoint_roundtrip(trained, tmp_path):
    import torch
    sur, _ = trained
    path = str(tmp_path / "sur.npz")
    sur.save(path)
    back = hs.Surrogate.load(path)
    assert back.step == sur.step and back.rmse_val == sur.rmse_val
    assert np.array_equal(back.wbf.cpu().numpy(), sur.wbf.cpu().numpy())
    _, x, _, y = _hybrid_case(sur, seed=2102, size=48)
    y2 = back.predict(x)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), y2.cpu().numpy())
