"""Seeded synthetic hyperspectral scenes with implanted sub-pixel anomalies.

The GPU tests, the oracle tests and the benchmark all take their inputs from this module.
It holds no arithmetic of the detection method: it builds cubes and truth masks only.

The paper evaluates on AVIRIS San Diego sub-images (Sec. 5.1).  That data is not
available here, so these scenes stand in for it.  They keep the paper's cube layout
(pixel vectors of L bands, Sec. 2.1) and its target-implant model, eq. (10):
z = f t + (1 - f) b.

Recipe (numpy PCG64, fully determined by the seed):

* K + 1 smooth spectra, the last one being the target.  Each is a sum of 6 Gaussian
  bumps over the band index: amplitude U(0.1, 1), centre U(0, L), width U(L/50, L/8).
* Background: a Gaussian-weighted mixture of the K endmembers.  Endmember k has a
  centre c_k ~ U(image) and a width s_k ~ U(0.15, 0.5) * min(H, W).  Its weight at
  pixel p is exp(-|p - c_k|^2 / (2 s_k^2)), normalised over k.
* Anomalies: single pixels and 2x2 blobs at uniform positions, with a Chebyshev
  distance > 2 between objects.  Each object draws one fraction f ~ U(0.3, 0.7) and
  every pixel of the object becomes f t + (1 - f) b  (eq. 10).
* Noise: i.i.d. N(0, noise^2) on every band, noise = 0.01 by default.
* Adjacency (eq. 11, optional, off by default): with adjacency_w = w > 0, every
  background pixel z_i within Chebyshev distance 1 of an object (the paper applies the
  effect "at a spatial distance of one") becomes
  exp(-rho_i^2 / w^2) f t + (1 - exp(-rho_i^2 / w^2) f) b_i, where rho_i is the Euclidean
  distance from z_i to the object's nearest pixel (1 for edge neighbours, sqrt(2) for
  corner neighbours) and f is the object's fraction.  Objects are more than 2 pixels
  apart, so no background pixel touches two objects.  It draws no random numbers, so a
  scene with the effect has the same spectra, objects, fractions and noise as without.
* Truth mask: 1 on anomaly pixels (the adjacency ring stays background).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Scene", "make_spectra", "make_scene", "make_scene_torch", "CONFIGS",
           "batch_scene_specs", "random_cube", "adjacency_ring"]


@dataclass
class Scene:
    cube: np.ndarray           # H x W x L float32, band fastest (BIP)
    truth: np.ndarray          # H x W uint8
    spectra: np.ndarray        # (K+1) x L float64, last row = target
    fractions: np.ndarray      # per-object f
    objects: list = field(default_factory=list)   # (y, x, size)


def make_spectra(rng: np.random.Generator, n: int, L: int, bumps: int = 6) -> np.ndarray:
    b = np.arange(L, dtype=np.float64)
    out = np.zeros((n, L))
    for i in range(n):
        A = rng.uniform(0.1, 1.0, bumps)
        c = rng.uniform(0.0, L, bumps)
        s = rng.uniform(L / 50.0, L / 8.0, bumps)
        out[i] = (A[:, None] * np.exp(-((b[None, :] - c[:, None]) ** 2) / (2 * s[:, None] ** 2))).sum(0)
    return out


def _place_objects(rng, H, W, n_single, n_blob, max_tries=200000):
    """Uniform positions, Chebyshev distance > 2 between object footprints."""
    taken = np.zeros((H, W), dtype=bool)
    objs = []
    sizes = [2] * n_blob + [1] * n_single
    tries = 0
    for sz in sizes:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("could not place %d objects in %dx%d" % (len(sizes), H, W))
            y = int(rng.integers(0, H - sz + 1))
            x = int(rng.integers(0, W - sz + 1))
            y0, y1 = max(0, y - 2), min(H, y + sz + 2)
            x0, x1 = max(0, x - 2), min(W, x + sz + 2)
            if not taken[y0:y1, x0:x1].any():
                taken[y:y + sz, x:x + sz] = True
                objs.append((y, x, sz))
                break
    return objs


def adjacency_ring(H: int, W: int, y: int, x: int, sz: int):
    """Background pixels at Chebyshev distance 1 from the sz x sz object at (y, x), with
    rho, the Euclidean distance to the object's nearest pixel: a list of (yy, xx, rho)."""
    out = []
    for yy in range(max(0, y - 1), min(H, y + sz + 1)):
        for xx in range(max(0, x - 1), min(W, x + sz + 1)):
            if y <= yy < y + sz and x <= xx < x + sz:
                continue
            dy = (y - yy) if yy < y else (yy - (y + sz - 1) if yy >= y + sz else 0)
            dx = (x - xx) if xx < x else (xx - (x + sz - 1) if xx >= x + sz else 0)
            out.append((yy, xx, float(np.hypot(dy, dx))))
    return out


def make_scene(seed: int, H: int, W: int, L: int, K: int = 8, n_single: int = 12,
               n_blob: int = 0, noise: float = 0.01, f_range=(0.3, 0.7),
               chunk_rows: int = 64, adjacency_w: float = 0.0) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    spectra = make_spectra(rng, K + 1, L)
    bg_spec, target = spectra[:K], spectra[K]
    m = min(H, W)
    centres = np.stack([rng.uniform(0, H, K), rng.uniform(0, W, K)], 1)
    widths = rng.uniform(0.15, 0.5, K) * m
    objs = _place_objects(rng, H, W, n_single, n_blob)
    fr = rng.uniform(f_range[0], f_range[1], len(objs))
    noise_rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(1)[0]))

    cube = np.empty((H, W, L), dtype=np.float32)
    xs = np.arange(W, dtype=np.float64)
    for r0 in range(0, H, chunk_rows):
        r1 = min(H, r0 + chunk_rows)
        ys = np.arange(r0, r1, dtype=np.float64)
        d2 = ((ys[:, None, None] - centres[None, None, :, 0]) ** 2
              + (xs[None, :, None] - centres[None, None, :, 1]) ** 2)
        logw = -d2 / (2.0 * widths[None, None, :] ** 2)
        logw -= logw.max(axis=2, keepdims=True)
        w = np.exp(logw)
        a = w / w.sum(axis=2, keepdims=True)
        bg = a @ bg_spec                                   # rows x W x L
        bg += noise_rng.normal(0.0, noise, bg.shape) if noise > 0 else 0.0
        cube[r0:r1] = bg.astype(np.float32)

    truth = np.zeros((H, W), dtype=np.uint8)
    for (y, x, sz), f in zip(objs, fr):
        blk = cube[y:y + sz, x:x + sz].astype(np.float64)
        cube[y:y + sz, x:x + sz] = (f * target + (1.0 - f) * blk).astype(np.float32)
        truth[y:y + sz, x:x + sz] = 1
        if adjacency_w > 0:
            for yy, xx, rho in adjacency_ring(H, W, y, x, sz):
                e = np.exp(-rho * rho / (adjacency_w * adjacency_w)) * f
                cube[yy, xx] = (e * target + (1.0 - e) * cube[yy, xx].astype(np.float64)).astype(np.float32)
    return Scene(cube=cube, truth=truth, spectra=spectra, fractions=fr, objects=objs)


def make_scene_torch(seed: int, H: int, W: int, L: int, K: int = 8, n_single: int = 12,
                     n_blob: int = 0, noise: float = 0.01, f_range=(0.3, 0.7),
                     device="cuda", chunk_rows: int = 256, adjacency_w: float = 0.0):
    """The same recipe as make_scene with the per-pixel arrays built by torch on `device`,
    for workloads of many gigabytes.  Spectra, endmember centres and widths, object
    positions and fractions come from the same numpy stream as make_scene, so for a given
    seed they are identical.  Only the noise differs: it comes from torch's generator
    seeded with `seed`.  The implants (eq. 10) and the adjacency ring (eq. 11) are applied
    to all objects at once by gathers and scatters on `device`.
    Returns (cube tensor H x W x L float32, truth uint8 numpy, spectra)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    spectra = make_spectra(rng, K + 1, L)
    m = min(H, W)
    centres = np.stack([rng.uniform(0, H, K), rng.uniform(0, W, K)], 1)
    widths = rng.uniform(0.15, 0.5, K) * m
    objs = _place_objects(rng, H, W, n_single, n_blob)
    fr = rng.uniform(f_range[0], f_range[1], len(objs))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    bg_spec = torch.from_numpy(spectra[:K]).to(device)
    target = torch.from_numpy(spectra[K]).to(device)
    cen = torch.from_numpy(centres).to(device)
    wid = torch.from_numpy(widths).to(device)
    cube = torch.empty((H, W, L), dtype=torch.float32, device=device)
    xs = torch.arange(W, dtype=torch.float64, device=device)
    for r0 in range(0, H, chunk_rows):
        r1 = min(H, r0 + chunk_rows)
        ys = torch.arange(r0, r1, dtype=torch.float64, device=device)
        d2 = (ys[:, None, None] - cen[None, None, :, 0]) ** 2 + (xs[None, :, None] - cen[None, None, :, 1]) ** 2
        logw = -d2 / (2.0 * wid[None, None, :] ** 2)
        logw = logw - logw.max(dim=2, keepdim=True).values
        w = torch.exp(logw)
        a = w / w.sum(dim=2, keepdim=True)
        bg = a @ bg_spec
        if noise > 0:
            bg += torch.randn(bg.shape, generator=gen, dtype=torch.float64, device=device) * noise
        cube[r0:r1] = bg.to(torch.float32)
    truth = np.zeros((H, W), dtype=np.uint8)
    # eq. (10) on every object pixel, eq. (11) on every ring pixel, as two batched updates
    # (objects are more than 2 pixels apart, so no pixel is written twice)
    pix, fpix, rpix, frng, erng = [], [], [], [], []
    for (y, x, sz), f in zip(objs, fr):
        for yy in range(y, y + sz):
            for xx in range(x, x + sz):
                pix.append(yy * W + xx)
                fpix.append(f)
        truth[y:y + sz, x:x + sz] = 1
        if adjacency_w > 0:
            for yy, xx, rho in adjacency_ring(H, W, y, x, sz):
                rpix.append(yy * W + xx)
                erng.append(np.exp(-rho * rho / (adjacency_w * adjacency_w)) * f)
    flat = cube.view(H * W, L)
    for ids, coef in ((pix, fpix), (rpix, erng)):
        if not ids:
            continue
        it = torch.tensor(ids, dtype=torch.int64, device=device)
        c = torch.tensor(coef, dtype=torch.float64, device=device)[:, None]
        b = flat.index_select(0, it).to(torch.float64)
        flat.index_copy_(0, it, (c * target[None, :] + (1.0 - c) * b).to(torch.float32))
    return cube, truth, spectra


def random_cube(seed: int, H: int, W: int, L: int, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) float32 cube (for shape/edge-case tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((H, W, L)) * scale).astype(np.float32)


# Named workloads.  Window sizes are (inner, outer); levels is the DWT depth.
CONFIGS = {
    # plain method, parity-sized
    "small_64x64x224": dict(seed=1201, H=64, W=64, L=224, K=4, n_single=12, n_blob=0, levels=6,
               inner=3, outer=9, load_rel=1e-6),
    # headline cube: levels 0 (full band) .. 6
    "cube_512x512x224": dict(seed=1202, H=512, W=512, L=224, K=8, n_single=150, n_blob=50, levels=6,
               inner=5, outer=15, load_rel=1e-6),
    # DWEST on the 512 x 512 x 224 cube at L' = 14 / 28 / 56
    "dwest_512x512x224": dict(seed=1202, H=512, W=512, L=224, K=8, n_single=150, n_blob=50,
               levels=(4, 3, 2), inner=3, outer=11),
    # surrogate: training scenes (seed 1205 + i) and the inference scene
    "surrogate_train_256x256x224": dict(seed=1205, H=256, W=256, L=224, K=8, n_single=40, n_blob=10,
                     levels=4, inner=5, outer=15, load_rel=1e-6, n_scenes=200),
    "surrogate_use_2048x2048x224": dict(seed=1299, H=2048, W=2048, L=224, K=8, n_single=2560, n_blob=640,
                     levels=4, inner=5, outer=15, load_rel=1e-6),
    # stand-ins for the paper's Img1 / Img2 shapes (Sec. 5.1, windows of Sec. 5.2)
    "img1_60x100x189": dict(seed=1301, H=60, W=100, L=189, K=6, n_single=10, n_blob=4, levels=5,
               lrx_inner=1, lrx_outer=15, inner=5, outer=13, load_rel=1e-6),
    "img2_100x100x189": dict(seed=1302, H=100, W=100, L=189, K=6, n_single=30, n_blob=2, levels=5,
               lrx_inner=1, lrx_outer=15, inner=3, outer=13, load_rel=1e-6),
}


def batch_scene_specs(seed: int = 1204, n: int = 64, hw=(128, 1024), L=(100, 430),
                      levels=(2, 5), outer=(9, 21), inner=(3, 7), K: int = 6):
    """Parameters of an uneven batch of scenes (one PCG64 stream per scene spawned from
    `seed`).  Objects scale with the area: about 200 per 512 x 512."""
    specs = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n)):
        r = np.random.Generator(np.random.PCG64(ss))
        H = int(r.integers(hw[0], hw[1] + 1))
        W = int(r.integers(hw[0], hw[1] + 1))
        Lb = int(r.integers(L[0], L[1] + 1))
        lv = int(r.integers(levels[0], levels[1] + 1))
        o = int(r.choice(np.arange(outer[0], outer[1] + 1, 2)))
        inn = int(r.choice([v for v in range(inner[0], inner[1] + 1, 2) if v < o]))
        nobj = max(4, int(round(H * W / 1311.0)))
        specs.append(dict(seed=int(ss.generate_state(1)[0]), H=H, W=W, L=Lb, K=K,
                          n_single=nobj - nobj // 4, n_blob=nobj // 4, levels=lv,
                          inner=inn, outer=o, load_rel=1e-6))
    return specs
