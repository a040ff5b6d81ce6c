"""Throughput of the DWT-reduced local anomaly detector on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--level J] [--no-sweep] [--no-cpu]

Workload: a 512 x 512 x 224 FP32 synthetic cube (8 endmembers, 200 implanted anomaly
objects including 2x2 blobs).  One step is the detection hot path over the cube:
  1. hsad_dwt        per-pixel db4 DWT to L' approximation coefficients (Sec. 4);
  2. hsad_detect     LRX (eq. 1) and DWRX (eq. 5) with a 5x5 inner / 15x15 outer window,
                     from one pass of window statistics, then the eq. (12) cut-off
                     tau = mu + 3 sigma of the LRX map and the anomaly mask.
The default depth is the paper's rule, "until four samples are left": J = 6, L' = 4.
Inputs are resident in HBM before timing.  Two copies of the cube alternate between
steps so that the 256 MB Infinity Cache cannot hold the input.  One JSON line is
printed.  Beside the timed step, the script also measures:
  * the same detector at full band (no DWT, L' = 224, exact FP64 Gram) on the same cube;
  * the DWT levels 1..5 sweep;
  * ROC AUC of the GPU scores minus that of the FP64 oracle scores (truth mask known);
  * the FP64 CPU oracle on the host cores, for the same workload (cpu_baseline);
  * the 64-scene uneven batch through the persistent batch engine;
  * DWEST (eqs. 2-4) at L' = 14 / 28 / 56 on the same cube (inner 3, outer 11);
  * the paper's image shapes and windows (60x100x189, 100x100x189), each detector with and without the DWT;
  * the learned surrogate: exact vs hybrid LRX on a 2048 x 2048 x 224 scene at L' = 14
    and 56, with the change of ROC AUC;
  * the reduced-precision Grams at L' = 56, global RX (eq. 1 over the whole image), the full
    DWT and its inverse (Daubechies orders 1, 4, 16), a Table 1-style AUC sweep with the eq. 11
    adjacency ring, and max / p99 / median errors of LRX, DWRX and DWEST against the oracle;
  * with --oracle-protocol, the FP64 oracle at 1 thread and all threads on every configuration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
FP64_PEAK = 78.6e12        # MI355X FP64, vector and matrix, flop/s


def annulus_samples(H, W, inner, outer):
    """Sum over all pixels of n_a, the annulus sample count with windows clipped at the image
    border (outer window minus inner window, Sec. 2.2)."""
    def clipped(n, r):
        c = np.arange(n)
        return np.minimum(c, r) + np.minimum(n - 1 - c, r) + 1
    ro, ri = outer // 2, inner // 2
    tot = clipped(H, ro).sum() * clipped(W, ro).sum()
    if inner > 0:
        tot -= clipped(H, ri).sum() * clipped(W, ri).sum()
    return float(tot)


def lrx_fp64_roofline(H, W, Lp, inner, outer, ms):
    """FP64 roofline of one LRX + DWRX call: the definition's flops, the annulus Gram
    (n_a L'(L'+1) per pixel: L'(L'+1)/2 entries, a multiply-add per sample each) plus the
    Cholesky and the two triangular solves (L'^3/3 + 2 L'^2 per pixel), over the call's time.
    The box-statistics path (L' <= 128) needs fewer flops than this definition count."""
    flops = annulus_samples(H, W, inner, outer) * Lp * (Lp + 1) + H * W * (Lp ** 3 / 3.0 + 2.0 * Lp ** 2)
    ach = flops / (ms * 1e-3)
    return {"bound": "fp64", "achieved": ach / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK, "flops": flops}
METRIC = "pixels/s for DWT+LRX at 512×512×224 vs full-band GPU; ROC AUC delta vs FP64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps first (the pipelined schedules reach their steady rate after ~300: "
                         "59 / 56 / 54 us per step after 10 / 100 / 300 at 512x512x224)")
    ap.add_argument("--level", type=int, default=None, help="DWT levels (default: paper rule)")
    ap.add_argument("--schedule", choices=("stream", "fused", "separate"), default="stream",
                    help="stream: each step is one hsad_detect_stream_step call (reduce the next cube, score "
                         "the current one, threshold the previous one, in one launch where L' <= 5 and "
                         "L %% 4 == 0); fused: one hsad_dwt_detect_fused call (reduce the next cube, score "
                         "and threshold the current one); separate: hsad_dwt then hsad_detect")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fullband", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-scene batch measurement")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--no-dwest", action="store_true", help="skip the DWEST measurement")
    ap.add_argument("--no-paper-shaped", action="store_true", help="skip the paper-shaped 60x100x189 and 100x100x189 runs")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate measurement")
    ap.add_argument("--surrogate-scenes", type=int, default=200,
                    help="training scenes of 256x256x224 for the surrogate (200 in the full workload)")
    ap.add_argument("--surrogate-levels", type=str, default="4,2",
                    help="DWT depths of the surrogate measurement (4 -> L'=14, 2 -> L'=56)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reduced-precision, global RX, full DWT, Table 1 sweep and error sections")
    ap.add_argument("--oracle-protocol", action="store_true",
                    help="also time the FP64 oracle, 1 thread and all threads, on every configuration (minutes)")
    ap.add_argument("--profile-workload", type=str, default=None,
                    help="run one named workload 3 times (after one warm-up) for a profiler and exit: "
                         "fullband, lp56, lp56_bf16, lp4, fused4, dwest14, dwest56, grx4, grx224, wavelet")
    ap.add_argument("--profile", action="store_true",
                    help="timed steps only, then 3 plain 256 MiB device copies (counter calibration)")
    return ap.parse_args()


def kernel_source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1201_2025_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, src_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(kernel, {}).get(workload)
        if not e or e.get("source_hash") != src_hash:
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def bench_batch(args, dev):
    """64 uneven synthetic scenes (H, W in [128, 1024], L in [100, 430], DWT depth 2..5,
    outer 9..21, inner 3..7) run by the persistent batch engine with an autotuned schedule.
    Returns a dict for the JSON line."""
    import torch
    import paper_1201_2025_amd as hs
    from paper_1201_2025_amd import synth
    specs = synth.batch_scene_specs(seed=1204, n=args.batch_scenes)
    scenes, cube_bytes, npix = [], 0, 0
    bound_s = 0.0
    for sp in specs:
        cube, _, _ = synth.make_scene_torch(sp["seed"], sp["H"], sp["W"], sp["L"], K=sp["K"],
                                            n_single=sp["n_single"], n_blob=sp["n_blob"], device=dev)
        scenes.append(dict(cube=cube, levels=sp["levels"], inner=sp["inner"], outer=sp["outer"],
                           load_rel=sp["load_rel"]))
        n = sp["H"] * sp["W"]
        Lp = hs.hsad_dwt_out_len(sp["L"], sp["levels"])
        npix += n
        cube_bytes += n * sp["L"] * 4
        # per-scene lower bound: max(HBM time, FP64 work of the Gram and Cholesky steps)
        hbm = n * (sp["L"] + Lp) * 4 / HBM_PEAK
        fp64 = 0.0
        if Lp > 8:
            T = (Lp + 15) // 16
            K = sp["outer"] ** 2
            fp64 = n * (T * (T + 1) / 2 * 256 * K * 2 + Lp ** 3 / 3) / 78.6e12
        bound_s += max(hbm, fp64)
    torch.cuda.synchronize()
    cache = os.environ.get("HSAD_TUNE_CACHE", os.path.join(ROOT, "_build", "hsad_tune.json"))
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    plan0 = hs.BatchPlan(scenes)                   # default schedule, also sizes the tables
    tune_ws = torch.empty(plan0.ws.numel() + (3 << 30), dtype=torch.uint8, device=dev)
    best, tune_ms = hs.hsad_batch_autotune(scenes, tune_ws, cache)
    del tune_ws
    plan0.close()
    plan = hs.BatchPlan(scenes, best)
    plan.run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    a.record()
    for _ in range(reps):
        plan.run()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    info = plan.info()
    plan.close()
    return {"workload": "%d uneven scenes, H,W in [128,1024], L in [100,430], levels 2-5, "
                        "outer 9-21, inner 3-7 (torch-generated, same recipe)" % len(specs),
            "pixels": npix, "cube_bytes": cube_bytes, "ms": ms, "pixels_per_s": npix / (ms * 1e-3),
            "bound_ms": bound_s * 1e3, "frac_of_bound": bound_s * 1e3 / ms,
            "schedule": {"wgs_per_cu": best.wgs_per_cu, "dwt_pixels": best.dwt_pixels,
                         "chunk_bytes": best.chunk_bytes, "tuning_ms": tune_ms},
            "plan": info}


def bench_dwest(cube, dev, log):
    """DWEST (eqs. 2-4) on the 512 x 512 x 224 cube reduced to L' = 14 / 28 / 56, inner 3 x 3,
    outer 11 x 11: FP64 box statistics of the inner and annulus windows, then per pixel a
    Householder tridiagonalisation of C_diff and the implicit QL iteration with m_diff carried
    through.  Reports time, pixels/s and the FP64 rate of the nominal 9 L'^3 flop per pixel
    of a symmetric eigensolve with vectors."""
    import torch
    import paper_1201_2025_amd as hs
    H, W = cube.shape[0], cube.shape[1]
    out = []
    for lv in (4, 3, 2):
        if out and out[-1]["ms"] > 2000.0:
            break
        x = hs.hsad_dwt(cube, lv)
        Lp = x.shape[2]
        ws = torch.empty(hs.hsad_workspace_bytes(hs.HSAD_OP_DWEST, H, W, Lp, 3, 11, 0.0), dtype=torch.uint8,
                         device=dev)
        hs.hsad_dwest(x, 3, 11, ws=ws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        hs.hsad_dwest(x, 3, 11, ws=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        nominal = 9.0 * Lp ** 3 * H * W
        out.append({"levels": lv, "Lp": Lp, "ms": ms, "pixels_per_s": H * W / (ms * 1e-3),
                    "nominal_fp64_tflops": nominal / (ms * 1e-3) / 1e12,
                    "roofline": {"bound": "fp64", "achieved": nominal / (ms * 1e-3) / 1e12,
                                 "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                                 "frac": nominal / (ms * 1e-3) / FP64_PEAK, "flops": nominal,
                                 "count": "nominal 9 L'^3 per pixel"}})
        log("dwest L'=%d: %.2f ms" % (Lp, ms))
        del ws
    return {"workload": "512x512x224 cube (150 singles + 50 blobs) at L' = 14/28/56, inner 3, outer 11", "levels": out}


def bench_paper_shaped(dev, log):
    """The paper's image shapes (Sec. 5.1: 60x100x189 and 100x100x189, J = 5 so L' = 6) with its
    windows (Sec. 5.2: LRX 15x15 single window; DWRX / DWEST 5x5 or 3x3 inside 13x13), on seeded
    stand-in scenes.  GPU times of each detector with and without the DWT, beside the paper's
    own IDL runtimes on Img2 (Table 2, i5-2410M), which are context only."""
    import torch
    import paper_1201_2025_amd as hs
    from paper_1201_2025_amd import synth
    table2_s = {"LRX": 713.674, "DWT-LRX": 17.071, "DWRX": 637.089, "DWT-DWRX": 19.318,
                "DWEST": 1091.173, "DWT-DWEST": 20.129}
    out = {"table2_img2_seconds_idl_cpu": table2_s, "scenes": {}}

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    for name in ("img1_60x100x189", "img2_100x100x189"):
        c = synth.CONFIGS[name]
        sc = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"],
                              n_blob=c["n_blob"])
        cube = torch.from_numpy(sc.cube).to(dev)
        res = {}
        for full in (True, False):
            tag = "" if full else "DWT-"

            def red():
                return cube if full else hs.hsad_dwt(cube, c["levels"])
            res[tag + "LRX"] = timed(lambda: hs.hsad_lrx(red(), c["lrx_inner"], c["lrx_outer"], c["load_rel"]))
            res[tag + "DWRX"] = timed(lambda: hs.hsad_dwrx(red(), c["inner"], c["outer"], c["load_rel"]))
            res[tag + "DWEST"] = timed(lambda: hs.hsad_dwest(red(), c["inner"], c["outer"]), reps=5)
        out["scenes"][name] = {"shape": [c["H"], c["W"], c["L"]], "levels": c["levels"], "ms": res}
        log("%s: %s" % (name, ", ".join("%s %.2f ms" % kv for kv in res.items())))
    return out


def bench_surrogate(args, dev, log):
    """Learned surrogate: trained on exact LRX of generated 256x256x224 scenes, then used on
    one 2048x2048x224 scene (same recipe).  For each DWT depth, the exact path (DWT + LRX +
    eq. 12 mask) and the hybrid path (DWT + hsad_surrogate_run: features, network, band +
    1% audit, exact recompute, fallback check, eq. 12 mask) are timed on the same cube, and
    the ROC AUC of both maps against the truth mask is computed by hsad_auc."""
    import torch
    import paper_1201_2025_amd as hs
    from paper_1201_2025_amd import synth
    ct, ci = synth.CONFIGS["surrogate_train_256x256x224"], synth.CONFIGS["surrogate_use_2048x2048x224"]
    inner, outer, load = ct["inner"], ct["outer"], ct["load_rel"]
    t0 = time.perf_counter()
    cube, truth, _ = synth.make_scene_torch(ci["seed"], ci["H"], ci["W"], 224, K=ci["K"],
                                            n_single=ci["n_single"], n_blob=ci["n_blob"], device=dev)
    truth_t = torch.from_numpy(truth.ravel()).to(dev)
    H, W = ci["H"], ci["W"]
    npix = H * W
    gen_s = time.perf_counter() - t0
    out = {"workload": "train: %d scenes 256x256x224 (seeds %d+i); use: 2048x2048x224 seed %d; "
                       "inner %d outer %d; band 3 x validation RMSE, 1%% audit, fallback at 2 x"
                       % (args.surrogate_scenes, ct["seed"], ci["seed"], inner, outer),
           "scene_gen_s": gen_s, "levels": []}

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    for lv in [int(v) for v in args.surrogate_levels.split(",") if v]:
        Lp = hs.hsad_dwt_out_len(224, lv)
        t0 = time.perf_counter()
        sur = hs.Surrogate(Lp, inner, outer, load, seed=lv)
        n_val = max(1, args.surrogate_scenes // 20)
        for i in range(args.surrogate_scenes):
            c, _, _ = synth.make_scene_torch(ct["seed"] + i, ct["H"], ct["W"], 224, K=ct["K"],
                                             n_single=ct["n_single"], n_blob=ct["n_blob"], device=dev)
            sur.add_scene(c, lv)
            del c
        torch.cuda.synchronize()
        label_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        hist = sur.fit(epochs=8, batch=16384, lr=2e-3, lr_final=1e-4, val_scenes=n_val, seed=lv)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        train_rows = int(sur.X_train.shape[0])
        sur.release()
        torch.cuda.empty_cache()

        approx = torch.empty((H, W, Lp), dtype=torch.float32, device=dev)
        exact = torch.empty((H, W), dtype=torch.float32, device=dev)
        emask = torch.empty((H, W), dtype=torch.uint8, device=dev)
        ws_b = hs.hsad_workspace_bytes(hs.HSAD_OP_LRX, H, W, Lp, inner, outer, load)
        ws = torch.empty(max(ws_b, 1), dtype=torch.uint8, device=dev)
        th_ws = torch.empty(hs.hsad_threshold_workspace_bytes(npix), dtype=torch.uint8, device=dev)
        th = torch.empty(4, dtype=torch.float64, device=dev)

        def run_exact():
            hs.hsad_dwt(cube, lv, out=approx)
            hs.hsad_lrx(approx, inner, outer, load, out=exact, ws=ws if ws_b else None)
            hs.hsad_threshold(exact, 3.0, stats=th, mask=emask, ws=th_ws)

        exact_ms = timed(run_exact)
        del ws
        sws = torch.empty(sur.workspace_bytes(H, W), dtype=torch.uint8, device=dev)
        hyb = torch.empty((H, W), dtype=torch.float32, device=dev)
        hmask = torch.empty((H, W), dtype=torch.uint8, device=dev)
        rep = {}

        def run_hybrid():
            hs.hsad_dwt(cube, lv, out=approx)
            _, _, r = sur.run(approx, z_alpha=3.0, band_k=3.0, audit_frac=0.01, fallback_factor=2.0,
                              seed=12345, ws=sws, scores=hyb, mask=hmask, exact_above=False)
            rep.update(r)

        hybrid_ms = timed(run_hybrid)
        a_e = hs.auc_from_counts(hs.hsad_auc(exact, truth_t))
        a_h = hs.auc_from_counts(hs.hsad_auc(hyb, truth_t))
        mm = int((emask != hmask).sum().item())
        # the same with every predicted detection recomputed exactly (the band extends upward)
        rep_up = {}

        def run_hybrid_up():
            hs.hsad_dwt(cube, lv, out=approx)
            _, _, r = sur.run(approx, z_alpha=3.0, band_k=3.0, audit_frac=0.01, fallback_factor=2.0,
                              seed=12345, ws=sws, scores=hyb, mask=hmask, exact_above=True)
            rep_up.update(r)

        hybrid_up_ms = timed(run_hybrid_up)
        a_u = hs.auc_from_counts(hs.hsad_auc(hyb, truth_t))
        mm_u = int((emask != hmask).sum().item())
        hs.hsad_dwt(cube, lv, out=approx)
        pred_ms = timed(lambda: sur.predict(approx))
        del sws
        entry = {"levels": lv, "Lp": Lp, "train_rows": train_rows, "label_gen_s": label_s,
                 "train_s": train_s, "epochs": len(hist), "val_rmse": sur.rmse_val,
                 "history": [[round(a, 5), round(b, 5)] for a, b in hist],
                 "exact_ms": exact_ms, "hybrid_ms": hybrid_ms, "features_and_network_ms": pred_ms,
                 "gain": exact_ms / hybrid_ms,
                 "exact_pixels_per_s": npix / (exact_ms * 1e-3), "hybrid_pixels_per_s": npix / (hybrid_ms * 1e-3),
                 "auc_exact": a_e, "auc_hybrid": a_h, "auc_delta": a_h - a_e,
                 "mask_mismatch": mm, "report": rep,
                 "exact_above": {"hybrid_ms": hybrid_up_ms, "gain": exact_ms / hybrid_up_ms, "auc_hybrid": a_u,
                                 "auc_delta": a_u - a_e, "mask_mismatch": mm_u, "report": rep_up}}
        log("surrogate L'=%d: exact %.2f ms, hybrid %.2f ms (gain %.2fx), dAUC %.2e, selected %.4f, fallback %d, "
            "mask mismatches %d; with exact detections: %.2f ms, dAUC %.2e, selected %.4f, mask mismatches %d"
            % (Lp, exact_ms, hybrid_ms, exact_ms / hybrid_ms, a_h - a_e, rep["selected"] / npix, rep["fallback"], mm,
               hybrid_up_ms, a_u - a_e, rep_up["selected"] / npix, mm_u))
        out["levels"].append(entry)
        del sur, approx, exact, hyb
        torch.cuda.empty_cache()
    return out


def _timed_ms(fn, reps=10):
    """Median of reps event-timed calls after one warm-up call."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def _err_stats(g, r):
    """max / p99 / median of the elementwise relative error with a floor of 1e-3 * median."""
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    fin = np.isfinite(r) & np.isfinite(g)
    floor = 1e-3 * np.median(np.abs(r[fin]))
    e = np.abs(g[fin] - r[fin]) / np.maximum(np.abs(r[fin]), floor)
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "median": float(np.median(e)),
            "n": int(fin.sum())}


def bench_reduced_precision(cube, truth, dev, log):
    """The reduced-precision Grams against the exact path at L' = 56 (J = 2) on the 512 x 512 x 224
    cube, 5 x 5 / 15 x 15 windows (200 annulus samples >= 2 L'): time, ROC AUC and the error
    against the exact GPU map."""
    import torch
    import paper_1201_2025_amd as hs
    H, W = cube.shape[0], cube.shape[1]
    x = hs.hsad_dwt(cube, 2)
    Lp = x.shape[-1]
    truth_t = torch.from_numpy(truth.ravel()).to(dev)
    out = {"workload": "512x512x224 cube, J = 2 (L' = 56), LRX inner 5 outer 15", "Lp": Lp, "modes": {}}
    ref = None
    for name, prec in (("fp64", hs.HSAD_PREC_AUTO), ("fp32", hs.HSAD_PREC_FP32), ("bf16", hs.HSAD_PREC_GRAM_BF16),
                       ("fp16", hs.HSAD_PREC_GRAM_FP16)):
        wsb = hs.hsad_workspace_bytes(hs.HSAD_OP_LRX, H, W, Lp, 5, 15, 1e-6, prec)
        ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)
        l = torch.empty((H, W), dtype=torch.float32, device=dev)
        ms = _timed_ms(lambda: hs.hsad_lrx(x, 5, 15, 1e-6, prec, out=l, ws=ws), reps=3)
        a = hs.auc_from_counts(hs.hsad_auc(l, truth_t))
        m = l.cpu().numpy()
        e = {"ms": ms, "auc": a}
        if ref is None:
            ref = (m, a)
        else:
            e["auc_delta_vs_fp64"] = a - ref[1]
            e["err_vs_fp64"] = _err_stats(m, ref[0])
        out["modes"][name] = e
        log("reduced precision %s L'=%d: %.2f ms, AUC %.5f" % (name, Lp, ms, a))
        del ws
    return out


def bench_global_rx(cube, dev, log):
    """Global RX (eq. 1, whole image as background) on the 512 x 512 x 224 cube at L' = 4 (J = 6)
    and at full band.  Bound: HBM at L' = 4 (reduced cube read twice, scores written); FP64
    at full band (symmetric Gram and triangular scoring, 2 N L'(L'+1) flop)."""
    import torch
    import paper_1201_2025_amd as hs
    H, W = cube.shape[0], cube.shape[1]
    n = H * W
    out = {"workload": "512x512x224 cube, J = 6 (L' = 4) and full band (L' = 224)", "levels": []}
    for lv in (6, 0):
        x = hs.hsad_dwt(cube, lv) if lv else cube
        Lp = x.shape[-1]
        ws = torch.empty(hs.hsad_global_rx_workspace_bytes(n, Lp), dtype=torch.uint8, device=dev)
        sc = torch.empty((H, W), dtype=torch.float32, device=dev)
        ms = _timed_ms(lambda: hs.hsad_global_rx(x, 1e-6, out=sc, ws=ws), reps=10)
        e = {"levels": lv, "Lp": Lp, "ms": ms, "pixels_per_s": n / (ms * 1e-3)}
        if Lp <= 16:
            e["hbm_bytes"] = n * (8 * Lp + 4)
            e["bound_ms"] = e["hbm_bytes"] / HBM_PEAK * 1e3
        else:
            e["fp64_flop"] = 2.0 * n * Lp * (Lp + 1)
            e["bound_ms"] = e["fp64_flop"] / 78.6e12 * 1e3
        e["frac_of_bound"] = e["bound_ms"] / ms
        out["levels"].append(e)
        log("global RX L'=%d: %.3f ms (%.3f of bound)" % (Lp, ms, e["frac_of_bound"]))
        del ws
    return out


def bench_wavelet_full(cube, dev, log):
    """Full DWT [a_J d_J ... d_1] and its inverse (Daubechies orders 1, 4, 16; J = 3) on the
    512 x 512 x 224 cube: time and the fraction of HBM bandwidth (cube read + coefficients
    written, or the reverse)."""
    import torch
    import paper_1201_2025_amd as hs
    H, W, L = cube.shape
    out = {"workload": "512x512x224 cube, J = 3", "orders": []}
    for order in (1, 4, 16):
        c = hs.hsad_dwt_full(cube, 3, order)
        y = torch.empty_like(cube)
        f = _timed_ms(lambda: hs.hsad_dwt_full(cube, 3, order, out=c), reps=5)
        i = _timed_ms(lambda: hs.hsad_idwt_full(c, L, 3, order, out=y), reps=5)
        by = H * W * (L + c.shape[-1]) * 4
        out["orders"].append({"order": order, "taps": 2 * order, "forward_ms": f, "inverse_ms": i,
                              "forward_hbm_frac": by / (f * 1e-3) / HBM_PEAK,
                              "inverse_hbm_frac": by / (i * 1e-3) / HBM_PEAK})
        log("full DWT db%d: forward %.3f ms, inverse %.3f ms" % (order, f, i))
        del c, y
    return out


def bench_table1(dev, log):
    """Table 1-style AUC sweep (Sec. 5.3.1) on device-generated scenes with eq. 10 implants and
    the eq. 11 adjacency ring (w = 1): the Img1-shaped 60 x 100 x 189 scene with the paper's
    windows (LRX 15 x 15 single window, DWRX / DWEST 5 x 5 in 13 x 13) at every depth, and the
    512 x 512 x 224 cube (LRX / DWRX, 5 x 5 / 15 x 15) at J = 0 and 2..6."""
    from paper_1201_2025_amd import sweep
    res = {"img1_60x100x189": sweep.table1_sweep(adjacency_w=1.0)}
    rows = sweep.table1_sweep(H=512, W=512, L=224, seed=1202, K=8, n_single=150, n_blob=50, adjacency_w=1.0,
                              levels=[0, 2, 3, 4, 5, 6], lrx_window=(5, 15), dual_window=(5, 15),
                              detectors=("LRX", "DWRX"))
    res["cube_512x512x224"] = rows
    for k, v in res.items():
        log("table1 %s: %s" % (k, ", ".join("%s J=%d %.4f" % (r["detector"], r["levels"], r["auc"]) for r in v)))
    return res


def bench_errors(cube, approx_fn, dev, log):
    """max / p99 / median relative errors of LRX, DWRX (headline configuration, every pixel)
    and DWEST (L' = 14, inner 3, outer 11, 20 000 sampled pixels) against the FP64 oracle on
    the same FP32 reduced cube."""
    import torch
    import oracle
    import paper_1201_2025_amd as hs
    out = {}
    x = approx_fn(6)
    l, d = hs.hsad_lrx_dwrx(x, 5, 15, 1e-6)
    xn = x.cpu().numpy().astype(np.float64)
    rl, rd = oracle.lrx_dwrx(xn, 5, 15, 1e-6)
    out["lrx_L4"] = _err_stats(l.cpu().numpy(), rl)
    out["dwrx_L4"] = _err_stats(d.cpu().numpy(), rd)
    x = approx_fn(4)
    sc, lit, _ = hs.hsad_dwest(x, 3, 11)
    torch.cuda.synchronize()
    H, W = x.shape[0], x.shape[1]
    idx = np.sort(np.random.default_rng(5).choice(H * W, 20000, replace=False))
    rs, rlit, _ = oracle.dwest(x.cpu().numpy().astype(np.float64), 3, 11, idx=idx)
    out["dwest_L14"] = _err_stats(sc.cpu().numpy().ravel()[idx], rs)
    out["dwest_literal_L14"] = _err_stats(lit.cpu().numpy().ravel()[idx], rlit)
    log("errors: " + ", ".join("%s max %.2e p99 %.2e" % (k, v["max"], v["p99"]) for k, v in out.items()))
    return out


def oracle_protocol(log):
    """The FP64 oracle on this host, 1 thread and all threads, median of 3, per configuration:
    the 64 x 64 x 224 parity scene, the 512 x 512 x 224 cube at every depth (LRX + DWRX, 5 / 15),
    DWEST at L' = 14 / 28 / 56 (3 / 11) and the Img1 / Img2-shaped scenes (all three detectors).
    Heavy configurations run on a block of whole rows chosen to take about a second and are
    scaled to the whole image (pixels are independent); each entry says which."""
    import platform
    import oracle
    from paper_1201_2025_amd import synth
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nthreads = oracle.set_threads(None)
    res = {"cpu_model": cpu_model, "threads_all": nthreads, "machine": platform.machine(), "configs": []}

    def med3(fn):
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    def run(name, cube, levels, work, px_per_row):
        H = cube.shape[0]
        # rows: grow the block until one all-thread pass takes about 0.3 s (or the whole image)
        rows = min(H, 8)
        while True:
            sub = np.ascontiguousarray(cube[:rows])
            t = time.perf_counter()
            work(sub, levels)
            dt = time.perf_counter() - t
            if dt > 0.3 or rows >= H:
                break
            rows = min(H, rows * 2)
        entry = {"config": name, "rows": rows, "of_rows": H, "scaled": rows < H}
        for tag, th in (("all", nthreads), ("one", 1)):
            oracle.set_threads(th)
            s = med3(lambda: work(sub, levels))
            entry["%s_thread_s" % tag] = s * H / rows
            entry["%s_thread_pixels_per_s" % tag] = rows * px_per_row / s
        oracle.set_threads(nthreads)
        res["configs"].append(entry)
        log("oracle %s: all %.3g s, one %.3g s (rows %d of %d)" % (name, entry["all_thread_s"],
                                                                   entry["one_thread_s"], rows, H))

    def lrx_work(inner, outer):
        def w(sub, lv):
            x = oracle.dwt_approx(sub, lv) if lv else sub.astype(np.float64)
            oracle.lrx_dwrx(x, inner, outer, 1e-6)
        return w

    def dwest_work(inner, outer):
        def w(sub, lv):
            x = oracle.dwt_approx(sub, lv) if lv else sub.astype(np.float64)
            oracle.dwest(x, inner, outer)
        return w

    c = synth.CONFIGS["small_64x64x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
    run("64x64x224 J=6 LRX+DWRX 3/9", s.cube, 6, lrx_work(3, 9), c["W"])
    c = synth.CONFIGS["cube_512x512x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
    for lv in (6, 5, 4, 3, 2, 1, 0):
        run("512x512x224 J=%d LRX+DWRX 5/15" % lv, s.cube, lv, lrx_work(5, 15), c["W"])
    for lv in (4, 3, 2):
        run("512x512x224 J=%d DWEST 3/11" % lv, s.cube, lv, dwest_work(3, 11), c["W"])
    for name in ("img1_60x100x189", "img2_100x100x189"):
        c = synth.CONFIGS[name]
        s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
        for lv in (c["levels"], 0):
            run("%s J=%d LRX %d/%d" % (name, lv, c["lrx_inner"], c["lrx_outer"]), s.cube, lv,
                lrx_work(c["lrx_inner"], c["lrx_outer"]), c["W"])
            run("%s J=%d DWEST %d/%d" % (name, lv, c["inner"], c["outer"]), s.cube, lv,
                dwest_work(c["inner"], c["outer"]), c["W"])
    return res


def profile_workload(name, dev):
    """One named workload on the 512 x 512 x 224 cube, for rocprofv3 kernel traces and counters."""
    import torch
    import paper_1201_2025_amd as hs
    from paper_1201_2025_amd import synth
    c = synth.CONFIGS["cube_512x512x224"]
    s = synth.make_scene(c["seed"], c["H"], c["W"], c["L"], K=c["K"], n_single=c["n_single"], n_blob=c["n_blob"])
    cube = torch.from_numpy(s.cube).to(dev)
    H, W = c["H"], c["W"]
    spare = {}
    works = {
        "fullband": (0, lambda x: hs.hsad_lrx_dwrx(x, 5, 15, 1e-6)),
        "lp56": (2, lambda x: hs.hsad_lrx_dwrx(x, 5, 15, 1e-6)),
        "lp56_bf16": (2, lambda x: hs.hsad_lrx_dwrx(x, 5, 15, 1e-6, hs.HSAD_PREC_GRAM_BF16)),
        "lp4": (6, lambda x: hs.hsad_detect(x, 5, 15, 1e-6, 3.0)),
        # the headline step's shared launch: the DWT of the cube beside the detector of x
        "fused4": (6, lambda x: hs.hsad_dwt_detect_fused(cube, 6, spare.setdefault("a", torch.empty_like(x)), x,
                                                         5, 15, 1e-6, 3.0)),
        "dwest14": (4, lambda x: hs.hsad_dwest(x, 3, 11)),
        "dwest56": (2, lambda x: hs.hsad_dwest(x, 3, 11)),
        "grx4": (6, lambda x: hs.hsad_global_rx(x, 1e-6)),
        "grx224": (0, lambda x: hs.hsad_global_rx(x, 1e-6)),
        "wavelet": (None, lambda x: hs.hsad_idwt_full(hs.hsad_dwt_full(x, 3, 4), 224, 3, 4)),
    }
    if name not in works:
        raise SystemExit("unknown workload %r (one of %s)" % (name, ", ".join(works)))
    lv, fn = works[name]
    x = cube if not lv else hs.hsad_dwt(cube, lv)
    for i in range(4):
        fn(x)
        torch.cuda.synchronize()
        print("profile workload %s: run %d done" % (name, i), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the workload is "
              "the whole cube on one GPU; --gpus must be 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1201_2025_amd as hs
    from paper_1201_2025_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.profile_workload:
        profile_workload(args.profile_workload, dev)
        return
    c = synth.CONFIGS["cube_512x512x224"]
    H, W, L = c["H"], c["W"], c["L"]
    J = hs.hsad_levels_for(L, 4) if args.level is None else args.level
    Lp = hs.hsad_dwt_out_len(L, J)
    inner, outer, load = c["inner"], c["outer"], c["load_rel"]
    scene = synth.make_scene(c["seed"], H, W, L, K=c["K"], n_single=c["n_single"],
                             n_blob=c["n_blob"])
    npix = H * W

    cubes = [torch.from_numpy(scene.cube).to(dev) for _ in range(2)]
    approx = torch.empty((H, W, Lp), dtype=torch.float32, device=dev)
    lrx = torch.empty((H, W), dtype=torch.float32, device=dev)
    dwrx = torch.empty((H, W), dtype=torch.float32, device=dev)
    mask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    det_ws = torch.empty(hs.hsad_detect_workspace_bytes(H, W, Lp, inner, outer, load), dtype=torch.uint8,
                         device=dev)
    th_out = torch.empty(4, dtype=torch.float64, device=dev)
    # The default schedule treats the run as a stream of cubes (the same scene, two resident
    # copies).  stream: a three-stage pipeline, step i reduces cube i + 1, scores cube i
    # (reduced by step i - 1) and thresholds cube i - 1 (scored by step i - 1), in one launch
    # where the stages can share one (hsad_detect_stream_step).  fused: step i reduces cube
    # i + 1 and scores and thresholds cube i (hsad_dwt_detect_fused: one shared launch, then
    # the merge and mask).  separate: hsad_dwt then hsad_detect.  Every step is one whole
    # DWT, one whole detection and one whole threshold + mask; the pipeline fill runs before
    # the timed steps.
    shareable = Lp <= 5 and L % 4 == 0
    sched = args.schedule if shareable else "separate"
    bufs = [torch.empty((H, W, Lp), dtype=torch.float32, device=dev) for _ in range(2)]
    smap = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(2)]
    sws = [torch.empty_like(det_ws) for _ in range(2)]

    def step_separate(i, ev=None):
        # ev: two events that the DWT's kernel dispatch itself records at its start and end
        # (hsad_dwt_timed), whose difference is the launch duration
        if ev is not None:
            hs.hsad_dwt_timed(cubes[i & 1], J, ev[0], ev[1], out=approx)
        else:
            hs.hsad_dwt(cubes[i & 1], J, out=approx)
        # LRX + DWRX, then eq. (12) on the LRX map and the mask, in one library call
        hs.hsad_detect(approx, inner, outer, load, 3.0, lrx=lrx, dwrx=dwrx, stats=th_out, mask=mask,
                       ws=det_ws)

    def step_fused(i, ev=None):
        # ev: events that the shared launch's dispatch records at its start and end
        hs.hsad_dwt_detect_fused(cubes[(i + 1) & 1], J, bufs[(i + 1) & 1], bufs[i & 1], inner, outer, load, 3.0,
                                 lrx=lrx, dwrx=dwrx, stats=th_out, mask=mask, ws=det_ws,
                                 start=ev[0] if ev else None, stop=ev[1] if ev else None)

    def step_stream(i, ev=None):
        hs.hsad_detect_stream_step(cubes[(i + 1) & 1], J, bufs[(i + 1) & 1], bufs[i & 1], inner, outer,
                                   smap[i & 1], sws[i & 1], dwrx=dwrx, prev_lrx=smap[(i + 1) & 1],
                                   prev_ws=sws[(i + 1) & 1], prev_stats=th_out, prev_mask=mask, load_rel=load,
                                   z_alpha=3.0, start=ev[0] if ev else None, stop=ev[1] if ev else None)

    step = {"stream": step_stream, "fused": step_fused, "separate": step_separate}[sched]
    # pipeline fill: cube 0 reduced before step 0 (for the stream also scored, and cube 1
    # reduced, before step 1)
    hs.hsad_dwt(cubes[0], J, out=bufs[0])
    if sched == "stream":
        hs.hsad_detect_stream_step(cubes[1], J, bufs[1], bufs[0], inner, outer, smap[0], sws[0], dwrx=dwrx,
                                   load_rel=load)
    i0 = 1 if sched == "stream" else 0
    for i in range(i0, i0 + args.warmup):
        step(i)
    torch.cuda.synchronize()
    # the dominant launch's duration (roofline) comes from the events that its dispatch
    # records in every EV_EVERY-th timed step
    EV_EVERY = 10
    evs = {i: [torch.cuda.Event(enable_timing=True) for _ in range(2)]
           for i in range(args.steps) if i % EV_EVERY == 0}
    for pair in evs.values():      # torch creates an event on its first record: before the timing
        for e in pair:
            e.record()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    ibase = i0 + args.warmup         # the pipeline's buffers continue from the warm-up steps
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for i in range(args.steps):
        step(ibase + i, evs.get(i))
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / args.steps
    launch_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs.values()]))
    value = npix / (ms_step * 1e-3)
    # the timed run's last step left the scores of its last cube and (stream) the threshold
    # and mask of the one before (the same scene)
    last = ibase + args.steps - 1
    fl = (smap[last & 1] if sched == "stream" else lrx).clone()
    fd, fs, fm = dwrx.clone(), th_out.clone(), mask.clone()
    # the separate schedule's step and its DWT / detection shares, from an instrumented pass
    # outside the timed region
    nsplit = min(args.steps, 50)
    step_separate(0)           # first calls load the kernels: not in the instrumented pass
    sev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nsplit)]
    for trip in sev:
        for e in trip:
            e.record()
    for i in range(nsplit):
        step_separate(i, sev[i])
        sev[i][2].record()
    torch.cuda.synchronize()
    dwt_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in sev]))
    det_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in sev]))
    sep_ms = float(np.mean([e[0].elapsed_time(e[2]) for e in sev]))
    if sched == "separate":
        dwt_ms = launch_ms
    else:
        # the pipelined schedule's outputs must equal the separate calls' bit for bit (the
        # instrumented pass above left those in lrx, dwrx, th_out, mask)
        if not (torch.equal(fl, lrx) and torch.equal(fd, dwrx) and torch.equal(fs, th_out) and torch.equal(fm, mask)):
            print("bench.py: the %s schedule's outputs differ from the separate calls'" % sched, file=sys.stderr)
            sys.exit(1)

    if args.profile:
        # plain copies of known size: what FETCH_SIZE / WRITE_SIZE read for 256 MiB moved
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.steps, "schedule": sched,
                          "ms_per_step": ms_step, "launch_ms": launch_ms, "dwt_ms": dwt_ms, "detect_ms": det_ms,
                          "separate_ms_per_step": sep_ms}))
        return

    # dominant kernel, bound by HBM.  Algorithmic bytes per launch of the DWT: read the cube
    # once (H W L 4) and write the approximation matrix (H W L' 4).  The shared launch adds
    # the detector's: read the reduced cube once (H W L' 4), write the two score maps
    # (H W 8) and one (count, mean, M2) partial per 32 x 16 tile; the stream's adds the
    # threshold's: read the earlier LRX map (H W 4) and its partials, write its mask (H W).
    dwt_bytes = npix * L * 4 + npix * Lp * 4
    ntiles = ((H + 15) // 16) * ((W + 31) // 32)
    fused_bytes = dwt_bytes + npix * Lp * 4 + npix * 8 + ntiles * 24
    stream_bytes = fused_bytes + npix * 5 + ntiles * 24
    if sched != "separate":
        kern = "dwt_box_fused_kernel"
        launch_bytes = stream_bytes if sched == "stream" else fused_bytes
        src_hash = kernel_source_hash(["box.hip", "dev_box.hpp", "dwt.hip", "dev_dwt.hpp", "dev_thr.hpp"])
        traffic = load_traffic(kern, "C2_L%d_J%d_%d_%d%s" % (L, J, inner, outer, "_thr" if sched == "stream" else ""),
                               src_hash)
    else:
        kern, launch_bytes = ("dwt_equiv_lds_kernel" if Lp <= 16 else "dwt_banded_kernel"), dwt_bytes
        src_hash = kernel_source_hash(["dwt.hip", "dev_dwt.hpp"])
        traffic = load_traffic(kern, "C2_L%d_J%d" % (L, J), src_hash)
    achieved = launch_bytes / (launch_ms * 1e-3)
    dwt_kern = "dwt_equiv_lds_kernel" if Lp <= 16 else "dwt_banded_kernel"

    # ROC AUC of the GPU scores vs the FP64 oracle scores on the same cube
    gl = lrx.cpu().numpy().ravel()
    gd = dwrx.cpu().numpy().ravel()
    result_extra = {}
    cpu = None
    try:
        import oracle
        threads = oracle.set_threads(None)
        t = time.perf_counter()
        ra = oracle.dwt_approx(scene.cube, J)
        rl, rd = oracle.lrx_dwrx(ra, inner, outer, load)
        tau_ref = oracle.threshold(rl, 3.0)
        ref_mask = oracle.mask(rl, tau_ref)
        cpu_s = time.perf_counter() - t
        auc_gpu, auc_ref = oracle.auc(gl, scene.truth), oracle.auc(rl, scene.truth)
        dauc_gpu, dauc_ref = oracle.auc(gd, scene.truth), oracle.auc(rd, scene.truth)
        rel = np.abs(gl - rl) / np.maximum(np.abs(rl), 1e-3 * np.median(np.abs(rl)))
        result_extra["auc"] = {"lrx_gpu": auc_gpu, "lrx_fp64": auc_ref, "lrx_delta": auc_gpu - auc_ref,
                               "dwrx_gpu": dauc_gpu, "dwrx_fp64": dauc_ref,
                               "dwrx_delta": dauc_gpu - dauc_ref,
                               "lrx_rel_err_max": float(rel.max()),
                               "lrx_rel_err_median": float(np.median(rel)),
                               "mask_mismatch": int((mask.cpu().numpy().ravel() != ref_mask).sum())}
        if not args.no_cpu:
            # whole-cube passes of the oracle until about 10 s of CPU work have been timed
            reps, spent = [], 0.0
            while spent < 10.0 and len(reps) < 200:
                t = time.perf_counter()
                ra = oracle.dwt_approx(scene.cube, J)
                r_l, _ = oracle.lrx_dwrx(ra, inner, outer, load)
                oracle.mask(r_l, oracle.threshold(r_l, 3.0))
                reps.append(time.perf_counter() - t)
                spent += reps[-1]
            cpu = {"value": npix * len(reps) / spent, "unit": "pixels/s", "cores": threads,
                   "kind": "oracle",
                   "sample": "%d passes over the whole 512x512x224 cube (DWT J=%d + LRX/DWRX + eq. 12 "
                             "mask), %.1f s" % (len(reps), J, spent)}
    except Exception as e:       # the oracle is test infrastructure; report, don't fail
        result_extra["oracle_error"] = repr(e)

    # full band on the GPU: the same detector on the raw cube (L' = 224), exact FP64 Gram
    full = None
    if not args.no_fullband:
        fb_ws_bytes = hs.hsad_workspace_bytes(hs.HSAD_OP_LRX_DWRX, H, W, L, inner, outer, load)
        fb_ws = torch.empty(fb_ws_bytes, dtype=torch.uint8, device=dev)
        fl = torch.empty((H, W), dtype=torch.float32, device=dev)
        fd = torch.empty((H, W), dtype=torch.float32, device=dev)
        res = {}
        for name, prec in (("fp64", hs.HSAD_PREC_AUTO),):
            hs.hsad_lrx_dwrx(cubes[0], inner, outer, load, prec, lrx=fl, dwrx=fd, ws=fb_ws)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            hs.hsad_lrx_dwrx(cubes[1], inner, outer, load, prec, lrx=fl, dwrx=fd, ws=fb_ws)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            fsc = fl.cpu().numpy().ravel()
            r = {"ms": ms, "value": npix / (ms * 1e-3), "roofline": lrx_fp64_roofline(H, W, L, inner, outer, ms)}
            try:
                import oracle
                r["auc_lrx"] = oracle.auc(fsc, scene.truth)
            except Exception:
                pass
            res[name] = r
        del fb_ws
        full = res
        full["speedup_dwt_vs_fullband_fp64"] = value / res["fp64"]["value"]
        full["note"] = ("the reduced-precision Grams are refused at full band (200 annulus samples < 2 L'); "
                        "see reduced_precision for them at L' = 56")

    sweep = []
    if not args.no_sweep:
        for j in range(1, 7):
            lpj = hs.hsad_dwt_out_len(L, j)
            apx = torch.empty((H, W, lpj), dtype=torch.float32, device=dev)
            wsb = hs.hsad_workspace_bytes(hs.HSAD_OP_LRX_DWRX, H, W, lpj, inner, outer, load)
            wsj = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
            sl = torch.empty((H, W), dtype=torch.float32, device=dev)
            sd = torch.empty((H, W), dtype=torch.float32, device=dev)
            n = 3 if lpj > 16 else 20
            for i in range(2):
                hs.hsad_dwt(cubes[i & 1], j, out=apx)
                hs.hsad_lrx_dwrx(apx, inner, outer, load, lrx=sl, dwrx=sd, ws=wsj if wsb else None)
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            dts, lts = [], []
            for i in range(n):
                e[0].record()
                hs.hsad_dwt(cubes[i & 1], j, out=apx)
                e[1].record()
                hs.hsad_lrx_dwrx(apx, inner, outer, load, lrx=sl, dwrx=sd, ws=wsj if wsb else None)
                e[2].record()
                torch.cuda.synchronize()
                dts.append(e[0].elapsed_time(e[1]))
                lts.append(e[1].elapsed_time(e[2]))
            dm, lm = float(np.mean(dts)), float(np.mean(lts))
            sweep.append({"levels": j, "Lp": lpj, "dwt_ms": dm, "lrx_dwrx_ms": lm,
                          "pixels_per_s": npix / ((dm + lm) * 1e-3),
                          "dwt_hbm_frac": (npix * (L + lpj) * 4) / (dm * 1e-3) / HBM_PEAK,
                          "lrx_dwrx_roofline": lrx_fp64_roofline(H, W, lpj, inner, outer, lm)})
            del wsj

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dwest = None
    if not args.no_dwest:
        try:
            dwest = bench_dwest(cubes[0], dev, log)
        except Exception as e:     # report, keep the headline line
            dwest = {"error": repr(e)}

    paper_shaped = None
    if not args.no_paper_shaped:
        try:
            paper_shaped = bench_paper_shaped(dev, log)
        except Exception as e:     # report, keep the headline line
            paper_shaped = {"error": repr(e)}

    surrogate = None
    if not args.no_surrogate:
        try:
            surrogate = bench_surrogate(args, dev, log)
        except Exception as e:     # report, keep the headline line
            surrogate = {"error": repr(e)}

    extras = {}
    if not args.no_extras:
        for key, fn in (("reduced_precision", lambda: bench_reduced_precision(cubes[0], scene.truth, dev, log)),
                        ("global_rx", lambda: bench_global_rx(cubes[0], dev, log)),
                        ("wavelet_full", lambda: bench_wavelet_full(cubes[0], dev, log)),
                        ("table1_sweep", lambda: bench_table1(dev, log)),
                        ("errors", lambda: bench_errors(cubes[0], lambda lv: hs.hsad_dwt(cubes[0], lv), dev, log))):
            try:
                extras[key] = fn()
            except Exception as e:     # report, keep the headline line
                extras[key] = {"error": repr(e)}
            torch.cuda.empty_cache()
    if args.oracle_protocol and cpu is not None:
        try:
            cpu["protocol"] = oracle_protocol(log)
        except Exception as e:
            cpu["protocol"] = {"error": repr(e)}

    batch = None
    if not args.no_batch:
        try:
            batch = bench_batch(args, dev)
        except Exception as e:     # report, keep the headline line
            batch = {"error": repr(e)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "512x512x224 FP32 cube; db4 DWT J=%d (L'=%d) + LRX/DWRX inner 5 "
                               "outer 15 + eq. 12 mask" % (J, Lp),
                   "H": H, "W": W, "L": L, "levels": J, "Lp": Lp, "inner": inner,
                   "outer": outer, "load_rel": load, "storage": "f32", "parallelism": "1 GPU"},
        "schedule": {"stream": "stream: one launch per step reduces cube i+1, scores cube i and thresholds "
                               "cube i-1 (two buffers per stage)",
                     "fused": "fused: one launch per step reduces cube i+1 and scores cube i (two reduced "
                              "buffers), then the eq. 12 merge and mask",
                     "separate": "separate: hsad_dwt, then hsad_detect"}[sched],
        "kernel_ms": {"launch": launch_ms, "launch_event_samples": len(evs), "dwt": dwt_ms, "detect": det_ms,
                      "separate_step": sep_ms},
        "wall_s_timed": wall,
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": traffic, "algorithmic_bytes_per_launch": launch_bytes,
                     "source_hash": src_hash},
        "dwt_roofline": {"bound": "hbm", "kernel": dwt_kern,
                         "achieved": dwt_bytes / (dwt_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": dwt_bytes / (dwt_ms * 1e-3) / HBM_PEAK,
                         "traffic": load_traffic(dwt_kern, "C2_L%d_J%d" % (L, J),
                                                 kernel_source_hash(["dwt.hip", "dev_dwt.hpp"])),
                         "algorithmic_bytes_per_launch": dwt_bytes},
        "cpu_baseline": cpu,
        "full_band_gpu": full,
        "sweep": sweep,
        "batch": batch,
        "dwest": dwest,
        "paper_shaped": paper_shaped,
        "surrogate": surrogate,
    }
    out.update(extras)
    out.update(result_extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
