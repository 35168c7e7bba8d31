"""Pins of the photometric-loss oracle (paper Sec. 3.3, Eq. loss): the window,
SSIM's closed form on constant images, SSIM(x, x) = 1, and finite differences
of the loss."""
import numpy as np

from oracle import losses


def test_window_is_a_normalised_gaussian():
    g = losses.window().numpy()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    assert np.allclose(g, g[::-1])
    t = np.arange(-5, 6)
    np.testing.assert_allclose(g / g[5], np.exp(-t * t / 4.5), rtol=1e-14)


def test_ssim_closed_form_on_constant_images():
    a, b = 0.3, 0.7
    x = np.full((24, 30, 3), a)
    y = np.full((24, 30, 3), b)
    import torch
    s = losses.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    # away from the zero-padded border: means a, b and no variance
    want = (2 * a * b + losses.C1) / (a * a + b * b + losses.C1)
    np.testing.assert_allclose(s[5:-5, 5:-5], want, rtol=1e-12)


def test_identical_images_have_zero_loss():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (20, 17, 3))
    L, g = losses.loss_and_grad(x, x)
    assert abs(L) < 1e-12
    # at a minimum of the SSIM term its gradient vanishes; the L1 kink gives 0 (sign(0))
    assert np.abs(g).max() < 1e-10


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (9, 12, 3))
    y = rng.uniform(0, 1, (9, 12, 3))
    L, g = losses.loss_and_grad(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (4, 5, 1), (8, 11, 2), (3, 0, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (losses.loss_and_grad(xp, y)[0] - losses.loss_and_grad(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 + 1e-5 * abs(g[idx]), (idx, fd, g[idx])
