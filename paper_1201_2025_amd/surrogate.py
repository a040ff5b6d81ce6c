"""Training and use of the learned LRX surrogate (driver code over the C ABI).

The surrogate is an addition to the paper's method: an MLP that predicts log1p of the LRX
score (eq. 1) of a pixel from features of its annulus, so that the exact detector only
runs on the pixels near the eq. (12) threshold and on a seeded audit sample.  Every
numerical step runs in libhsad's kernels:
  labels     hsad_dwt + hsad_lrx (exact FP64 path) on each training scene,
  features   hsad_surrogate_features, normalised by hsad_mlp_norm_stats / hsad_mlp_pack,
  training   hsad_mlp_train_step (BF16 matrix-core forward/backward, FP32 Adam),
  validation hsad_mlp_infer + hsad_error_stats,
  use        hsad_surrogate_run (prediction, band + audit selection, exact recompute,
             fallback, eq. 12 mask).
This module only holds the tensors, draws the seeded initial weights and the epoch
permutations, and loops.
"""
from __future__ import annotations

import math

import numpy as np

from . import _binding as B

HID = 128


class Surrogate:
    """Model state: FP32 parameters, BF16 copy, Adam moments, input normalisation and the
    validation RMSE (log1p space), for L' reduced bands and one window pair."""

    def __init__(self, Lp: int, inner: int, outer: int, load_rel: float = 1e-6, seed: int = 0,
                 device: str = "cuda"):
        import torch
        self.Lp, self.inner, self.outer, self.load_rel = int(Lp), int(inner), int(outer), float(load_rel)
        self.D, self.Dp, self.nparams, self.nbf = B.hsad_mlp_dims(self.Lp)
        self.device = device
        self.params = torch.from_numpy(self._init_params(seed)).to(device)
        self.wbf = torch.empty(self.nbf, dtype=torch.int16, device=device)
        B.hsad_mlp_sync(self.params, self.Dp, self.wbf)
        self.m = torch.zeros(self.nparams, dtype=torch.float32, device=device)
        self.v = torch.zeros(self.nparams, dtype=torch.float32, device=device)
        self.norm = None
        self.step = 0
        self.rmse_val = None
        self._feat, self._tgt, self._scene_rows = [], [], []

    # ---- initial weights (He-normal for the ReLU layers), seeded ----
    def _init_params(self, seed: int) -> np.ndarray:
        r = np.random.Generator(np.random.PCG64(seed))
        D, Dp = self.D, self.Dp
        W1 = np.zeros((Dp, HID))
        W1[:D] = r.standard_normal((D, HID)) * math.sqrt(2.0 / D)
        W2 = r.standard_normal((HID, HID)) * math.sqrt(2.0 / HID)
        w3 = r.standard_normal(HID) * math.sqrt(1.0 / HID)
        p = np.concatenate([W1.ravel(), np.zeros(HID), W2.ravel(), np.zeros(HID), w3, np.zeros(4)])
        assert p.size == self.nparams
        return p.astype(np.float32)

    # ---- training data ----
    def add_scene(self, cube, levels: int):
        """Exact labels and FP32 features of one training scene (cube: H x W x L GPU tensor)."""
        x = B.hsad_dwt(cube, levels)
        if x.shape[2] != self.Lp:
            raise ValueError("scene reduces to L'=%d, model expects %d" % (x.shape[2], self.Lp))
        lrx = B.hsad_lrx(x, self.inner, self.outer, self.load_rel)
        self._tgt.append(B.hsad_surrogate_targets(lrx))
        self._feat.append(B.hsad_surrogate_features(x, self.inner, self.outer))
        self._scene_rows.append(x.shape[0] * x.shape[1])
        return x, lrx

    def fit(self, epochs: int = 8, batch: int = 16384, lr: float = 2e-3, lr_final: float = 1e-4,
            val_scenes: int = 1, seed: int = 0, log=None):
        """Trains on the scenes added so far; the last `val_scenes` scenes are held out for the
        validation RMSE, and the weights of the epoch with the lowest validation RMSE are kept
        (early stopping).  Returns the list of per-epoch (train loss, validation RMSE)."""
        import torch
        if len(self._feat) <= val_scenes:
            raise ValueError("need more training scenes than validation scenes")
        feat = torch.cat(self._feat)
        tgt = torch.cat(self._tgt)
        n_val = sum(self._scene_rows[-val_scenes:]) if val_scenes else 0
        n_tr = feat.shape[0] - n_val
        self.norm = B.hsad_mlp_norm_stats(feat[:n_tr].contiguous())
        X = B.hsad_mlp_pack(feat, self.norm, self.Dp)
        del feat
        self._feat = []
        # output bias starts at the mean training target (column statistics kernel)
        tstat = B.hsad_mlp_norm_stats(tgt[:n_tr].reshape(-1, 1).contiguous())
        off_b3 = self.Dp * HID + 3 * HID + HID * HID
        self.params[off_b3] = torch.nan_to_num(tstat[0], nan=0.0)
        B.hsad_mlp_sync(self.params, self.Dp, self.wbf)
        gen = torch.Generator(device=self.device)
        gen.manual_seed(int(seed))
        steps_per_epoch = max(1, n_tr // batch)
        total = epochs * steps_per_epoch
        ws = torch.empty(B.hsad_mlp_train_workspace_bytes(batch, self.Dp), dtype=torch.uint8, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        hist = []
        yv = torch.empty(max(n_val, 1), dtype=torch.float32, device=self.device)
        best, best_params = float("inf"), None
        k = 0
        for ep in range(epochs):
            perm = torch.randperm(n_tr, generator=gen, device=self.device).to(torch.int32)
            acc = torch.zeros((), dtype=torch.float64, device=self.device)
            for s in range(steps_per_epoch):
                rows = perm[s * batch:(s + 1) * batch]
                lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(1, total - 1)))
                self.step += 1
                k += 1
                B.hsad_mlp_train_step(X, tgt, rows, self.params, self.wbf, self.m, self.v, self.step, lr_k,
                                      loss=loss, ws=ws)
                acc += loss[0]
            rm = float("nan")
            if n_val:
                B.hsad_mlp_infer(X[n_tr:], self.params, self.wbf, out=yv)
                rm = float(B.hsad_error_stats(yv, tgt[n_tr:], False)[1])
            hist.append((float(acc) / steps_per_epoch, rm))
            if log:
                log("epoch %d loss %.5f val_rmse %.5f" % (ep, hist[-1][0], rm))
            if n_val and rm < best:          # early stopping: keep the best validated weights
                best, best_params = rm, self.params.clone()
        if best_params is not None:
            self.params.copy_(best_params)
            B.hsad_mlp_sync(self.params, self.Dp, self.wbf)
        self.rmse_val = best if n_val else None
        self._tgt, self._scene_rows = [], []
        self.X_train, self.tgt_train = X, tgt   # kept for inspection; dropped by release()
        return hist

    def release(self):
        self.X_train = self.tgt_train = None

    # ---- use ----
    def predict(self, x):
        """log1p(LRX) predictions of every pixel of the reduced cube x (H x W x L')."""
        Xp = B.hsad_surrogate_features(x, self.inner, self.outer, norm=self.norm, Dp=self.Dp)
        return B.hsad_mlp_infer(Xp, self.params, self.wbf).reshape(x.shape[0], x.shape[1])

    def run(self, x, z_alpha: float = 3.0, band_k: float = 3.0, audit_frac: float = 0.01,
            fallback_factor: float = 2.0, seed: int = 0, ws=None, scores=None, mask=True,
            band_quantile: float = 0.999, max_exact_frac: float = 0.25, exact_above: bool = True):
        """Hybrid LRX map of the reduced cube x: (scores, mask, report)."""
        if self.norm is None or self.rmse_val is None:
            raise RuntimeError("the surrogate is not trained")
        return B.hsad_surrogate_run(x, self.inner, self.outer, self.load_rel, self.params, self.wbf, self.norm,
                                    self.rmse_val, z_alpha=z_alpha, band_k=band_k, audit_frac=audit_frac,
                                    fallback_factor=fallback_factor, seed=seed, scores=scores, mask=mask, ws=ws,
                                    band_quantile=band_quantile, max_exact_frac=max_exact_frac,
                                    exact_above=exact_above)

    def workspace_bytes(self, H: int, W: int) -> int:
        return B.hsad_surrogate_workspace_bytes(H, W, self.Lp, self.Dp, self.inner, self.outer, self.load_rel)

    # ---- checkpoint ----
    def save(self, path: str):
        np.savez(path, Lp=self.Lp, inner=self.inner, outer=self.outer, load_rel=self.load_rel,
                 params=self.params.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 norm=self.norm.cpu().numpy() if self.norm is not None else np.zeros(0, np.float32),
                 step=self.step, rmse_val=np.nan if self.rmse_val is None else self.rmse_val)

    @classmethod
    def load(cls, path: str, device: str = "cuda"):
        import torch
        z = np.load(path, allow_pickle=False)
        s = cls(int(z["Lp"]), int(z["inner"]), int(z["outer"]), float(z["load_rel"]), device=device)
        s.params.copy_(torch.from_numpy(z["params"]))
        s.m.copy_(torch.from_numpy(z["m"]))
        s.v.copy_(torch.from_numpy(z["v"]))
        B.hsad_mlp_sync(s.params, s.Dp, s.wbf)
        s.norm = torch.from_numpy(z["norm"]).to(device) if z["norm"].size else None
        s.step = int(z["step"])
        r = float(z["rmse_val"])
        s.rmse_val = None if math.isnan(r) else r
        return s
