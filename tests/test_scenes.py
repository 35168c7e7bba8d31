"""The seeded input generator: reproducible bytes and the stated distributions."""
import math

import numpy as np

from paper_2411_14974_amd import scenes


def test_seeded_reproducible():
    a, ca, ta = scenes.config2(n=2000, width=64, height=48)
    b, cb, tb = scenes.config2(n=2000, width=64, height=48)
    for f in ("points", "delta", "sigma", "opacity", "sh"):
        assert getattr(a, f).tobytes() == getattr(b, f).tobytes()
    assert ca.R.tobytes() == cb.R.tobytes() and ta.tobytes() == tb.tobytes()
    c, _, _ = scenes.config2(variant=1, n=2000, width=64, height=48)
    assert c.points.tobytes() != a.points.tobytes()


def test_distributions():
    s, cam = scenes.config1()
    assert s.points.shape == (1000, 6, 3) and s.sh.shape == (1000, 1, 3) and s.deg == 0
    assert s.points.dtype == np.float32
    assert 1.0 <= s.delta.min() and s.delta.max() <= 50.0
    assert 1.0 <= s.sigma.min() and s.sigma.max() <= 20.0
    assert 0.1 <= s.opacity.min() and s.opacity.max() <= 0.9
    assert np.abs(s.sh).max() <= math.sqrt(math.pi) + 1e-6
    ctr = s.points.mean(1)
    assert ctr[:, 2].min() > 1.5 and ctr[:, 2].max() < 6.5
    assert cam.width == 128 and cam.fx == 128.0 and cam.cx == 64.0


def test_orbit_camera_is_a_rotation_looking_at_origin():
    rng = np.random.default_rng(0)
    for _ in range(20):
        cam = scenes.orbit_camera(rng, 640, 480)
        R = cam.R.astype(np.float64)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
        assert np.linalg.det(R) > 0.999
        campos = -R.T @ cam.t
        assert abs(np.linalg.norm(campos) - 4.0) < 1e-5
        # the origin projects onto the principal point, in front of the camera
        X = R @ np.zeros(3) + cam.t
        assert X[2] > 3.99 and abs(X[0]) < 1e-5 and abs(X[1]) < 1e-5


def test_mixture_and_serving_shapes():
    s, cam, tgt = scenes.config3(n=5000, width=96, height=54)
    assert s.n == 5000 and s.sh.shape == (5000, 16, 3) and tgt.shape == (54, 96, 3)
    reqs = scenes.serve_requests(rate=100.0, duration_s=1.0)
    assert 60 < len(reqs) < 140
    assert all(0 <= sid < 4 for _, sid, _ in reqs)
    assert all(r[0] < 1.0 for r in reqs) and all(reqs[i][0] < reqs[i + 1][0] for i in range(len(reqs) - 1))


def test_16bit_storage_rounding_matches_torch():
    """round_to is IEEE round-to-nearest-even into binary16 / bfloat16, bit for
    bit as torch converts (ties and signed zeros included)."""
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 3, 50000), rng.uniform(-60, 60, 50000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -1 - 2 ** -8, 1 + 2 ** -11, 1 + 3 * 2 ** -11,
                         0.0, -0.0, 50.0, 1e-30]]).astype(np.float32)
    for fmt, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        a = scenes.round_to(x, fmt)
        b = torch.from_numpy(x).to(dt).float().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), fmt
    # representable values are kept; a tie goes to the even neighbour
    assert scenes.round_to(np.float32(1 + 2 ** -7), "bf16") == np.float32(1 + 2 ** -7)
    assert scenes.round_to(np.float32(1 + 2 ** -8), "bf16") == np.float32(1.0)
    assert scenes.round_to(np.float32(1 + 3 * 2 ** -8), "bf16") == np.float32(1 + 2 ** -6)
    s, _ = scenes.config1()
    assert s.stored("f32") is s
    h = s.stored("f16")
    assert np.array_equal(h.points, s.points.astype(np.float16).astype(np.float32))
