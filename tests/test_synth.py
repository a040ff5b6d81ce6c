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
