"""The seeded scene generator: determinism, truth masks and the implant model (eq. 10)."""
import numpy as np

from paper_1201_2025_amd import synth


def test_deterministic_and_shapes():
    a = synth.make_scene(7, 20, 30, 50, K=3, n_single=5, n_blob=2)
    b = synth.make_scene(7, 20, 30, 50, K=3, n_single=5, n_blob=2)
    assert a.cube.shape == (20, 30, 50) and a.cube.dtype == np.float32
    assert np.array_equal(a.cube, b.cube) and np.array_equal(a.truth, b.truth)
    assert a.truth.sum() == 5 + 4 * 2
    assert len(a.objects) == 7 and np.all((a.fractions >= 0.3) & (a.fractions <= 0.7))


def test_implant_is_eq10_mixture():
    # without noise, an implanted pixel is f t + (1 - f) b with b the background there
    s = synth.make_scene(3, 16, 16, 40, K=2, n_single=3, noise=0.0)
    t = s.spectra[-1]
    for (y, x, sz), f in zip(s.objects, s.fractions):
        z = s.cube[y, x].astype(np.float64)
        # z - f t = (1 - f) b  with b a convex combination of the K background spectra
        bp = (z - f * t) / (1 - f)
        coef, *_ = np.linalg.lstsq(s.spectra[:-1].T, bp, rcond=None)
        assert np.allclose(s.spectra[:-1].T @ coef, bp, atol=1e-5)
        assert abs(coef.sum() - 1.0) < 1e-4 and np.all(coef > -1e-5)


def test_objects_are_separated():
    s = synth.make_scene(11, 64, 64, 8, K=2, n_single=40, n_blob=10)
    boxes = [(y, x, sz) for y, x, sz in s.objects]
    for i, (y1, x1, s1) in enumerate(boxes):
        for y2, x2, s2 in boxes[i + 1:]:
            gap_y = max(y2 - (y1 + s1 - 1), y1 - (y2 + s2 - 1))
            gap_x = max(x2 - (x1 + s1 - 1), x1 - (x2 + s2 - 1))
            assert max(gap_y, gap_x) > 2


def test_batch_specs():
    sp = synth.batch_scene_specs(n=16)
    assert len(sp) == 16
    for d in sp:
        assert 128 <= d["H"] <= 1024 and 100 <= d["L"] <= 430 and 2 <= d["levels"] <= 5
        assert d["inner"] < d["outer"] and d["outer"] % 2 == 1 and d["inner"] % 2 == 1


def test_adjacency_eq11_ring():
    """eq. (11): a background pixel next to an object becomes e f t + (1 - e f) b with
    e = exp(-rho^2 / w^2); nothing else changes, and no random number is drawn."""
    kw = dict(K=3, n_single=6, n_blob=3, noise=0.0)
    a = synth.make_scene(5, 24, 28, 30, **kw)
    w = 1.3
    b = synth.make_scene(5, 24, 28, 30, adjacency_w=w, **kw)
    assert a.objects == b.objects and np.array_equal(a.fractions, b.fractions)
    assert np.array_equal(a.truth, b.truth)
    t = a.spectra[-1]
    ring = np.zeros((24, 28), dtype=bool)
    for (y, x, sz), f in zip(a.objects, a.fractions):
        for yy, xx, rho in synth.adjacency_ring(24, 28, y, x, sz):
            assert not a.truth[yy, xx]
            # distance to the object's nearest pixel, by brute force over its pixels
            d = min(np.hypot(yy - py, xx - px) for py in range(y, y + sz) for px in range(x, x + sz))
            assert abs(d - rho) < 1e-12 and d in (1.0, np.sqrt(2.0))
            e = np.exp(-rho * rho / (w * w)) * f
            want = e * t + (1 - e) * a.cube[yy, xx].astype(np.float64)
            assert np.allclose(b.cube[yy, xx], want, rtol=1e-6, atol=1e-7)
            ring[yy, xx] = True
    assert ring.sum() >= 6 * 5 and not np.any(ring & (a.truth == 1))
    assert np.array_equal(a.cube[~ring], b.cube[~ring])
    # with noise the ring mixes the noisy background, the rest of the cube is unchanged
    c = synth.make_scene(5, 24, 28, 30, K=3, n_single=6, n_blob=3)
    d = synth.make_scene(5, 24, 28, 30, K=3, n_single=6, n_blob=3, adjacency_w=w)
    assert np.array_equal(c.cube[~ring], d.cube[~ring])


def test_adjacency_ring_corner_cases():
    # a 2 x 2 object has 12 ring pixels (8 edge, 4 corner); a single pixel has 8 (4 + 4);
    # at the image corner the ring is clipped
    r2 = synth.adjacency_ring(10, 10, 4, 4, 2)
    assert len(r2) == 12 and sorted(round(v, 6) for *_, v in r2).count(1.0) == 8
    r1 = synth.adjacency_ring(10, 10, 4, 4, 1)
    assert len(r1) == 8
    r0 = synth.adjacency_ring(10, 10, 0, 0, 1)
    assert sorted((yy, xx) for yy, xx, _ in r0) == [(0, 1), (1, 0), (1, 1)]


def test_torch_generator_matches_numpy_without_noise():
    """The torch form (run here on the CPU) builds the same cube as the numpy form when
    there is no noise, implants and adjacency ring included."""
    import torch
    for w in (0.0, 1.0):
        a = synth.make_scene(9, 20, 22, 17, K=3, n_single=5, n_blob=2, noise=0.0, adjacency_w=w)
        cube, truth, spectra = synth.make_scene_torch(9, 20, 22, 17, K=3, n_single=5, n_blob=2, noise=0.0,
                                                      device="cpu", adjacency_w=w)
        assert isinstance(cube, torch.Tensor)
        assert np.array_equal(truth, a.truth) and np.array_equal(spectra, a.spectra)
        assert np.allclose(cube.numpy(), a.cube, rtol=2e-7, atol=1e-7)
