"""Table 1-style detection sweeps on synthetic scenes, entirely on the GPU.

Sec. 5.3.1 compares the detectors by the area under their pixel-level ROC curves on an image
with implanted targets (Sec. 5.1.1: eq. 10 for the target pixels, eq. 11 for the background
pixels next to them).  ``table1_sweep`` repeats that comparison over DWT depths and window
pairs: the scene is generated on the device (``synth.make_scene_torch``, eqs. 10 and 11),
every detector runs through the library (LRX eq. 1, DWRX eq. 5, DWEST eqs. 2-4, on the full
band and after the DWT of Sec. 4), and each AUC comes from the library's exact pair counts
(``hsad_auc``).  Only the bookkeeping is Python; every pass over pixels is a library kernel.
"""
from __future__ import annotations

import time

from . import _binding as B
from . import synth

DETECTORS = ("LRX", "DWRX", "DWEST")


def _auc(scores, truth_t):
    import torch
    s = torch.nan_to_num(scores.contiguous(), nan=0.0, posinf=3.0e38, neginf=-3.0e38)
    return B.auc_from_counts(B.hsad_auc(s, truth_t).cpu())


def table1_sweep(H: int = 60, W: int = 100, L: int = 189, seed: int = 1301, K: int = 6, n_single: int = 10,
                 n_blob: int = 4, adjacency_w: float = 1.0, levels=None, lrx_window=(1, 15),
                 dual_window=(5, 13), detectors=DETECTORS, load_rel: float = 1e-6, device: str = "cuda",
                 scene=None, return_maps: bool = False):
    """AUC of every detector at every DWT depth on one synthetic scene.

    levels: DWT depths to run (0 = the full band; default 0 and every depth down to the
    paper's "four samples left", Sec. 4).  lrx_window: (inner, outer) of LRX (the paper's
    single 15 x 15 window excludes only the pixel, inner = 1).  dual_window: (inner, outer)
    of DWRX and DWEST.  scene: optional (cube tensor, truth uint8 array) to use instead of
    generating one.  Returns a list of rows {detector, levels, Lp, inner, outer, auc, ms}
    (with return_maps, each row also holds its score map as a device tensor under "map").
    """
    import torch
    if scene is None:
        cube, truth, _ = synth.make_scene_torch(seed, H, W, L, K=K, n_single=n_single, n_blob=n_blob,
                                                device=device, adjacency_w=adjacency_w)
    else:
        cube, truth = scene
        H, W, L = cube.shape
    truth_t = torch.as_tensor(truth, dtype=torch.uint8, device=cube.device).contiguous()
    if levels is None:
        levels = list(range(0, B.hsad_levels_for(L) + 1))
    rows = []
    for lv in levels:
        x = B.hsad_dwt(cube, lv) if lv else cube
        Lp = int(x.shape[-1])
        for det in detectors:
            inner, outer = lrx_window if det == "LRX" else dual_window
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if det == "LRX":
                s, _ = B.hsad_lrx_dwrx(x, inner, outer, load_rel, lrx=True, dwrx=False)
            elif det == "DWRX":
                _, s = B.hsad_lrx_dwrx(x, inner, outer, load_rel, lrx=False, dwrx=True)
            elif det == "DWEST":
                s, _, _ = B.hsad_dwest(x, inner, outer, literal=False, npos=False)
            else:
                raise ValueError("unknown detector %r" % det)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            row = dict(detector=det, levels=int(lv), Lp=Lp, inner=int(inner), outer=int(outer),
                       auc=_auc(s, truth_t), ms=ms)
            if return_maps:
                row["map"] = s
            rows.append(row)
    return rows
