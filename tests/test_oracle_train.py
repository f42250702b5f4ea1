"""Pins of the training-step reference (oracle/train.py): the loss of Sec. 5's
implementation details (l1 + 0.2 D-SSIM) and the Adam update, checked
against closed forms, invariants, finite differences and an independent
library implementation of Adam."""
import numpy as np
import pytest
import torch

from oracle import train as T


def test_window_is_a_normalised_gaussian():
    g = T.gaussian_window()
    assert g.shape == (11,)
    assert abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    # neighbouring taps differ by the Gaussian ratio exp((2k + 1) / (2 sigma^2))
    for k in range(5):
        assert np.isclose(g[5 + k] / g[6 + k], np.exp((2 * k + 1) / (2 * 1.5 ** 2)), rtol=1e-13)


def test_filter_is_zero_padded_and_separable():
    g = T.gaussian_window()
    img = np.zeros((15, 17))
    img[3, 4] = 1.0
    out = T.filter2(img, g)
    # an impulse spreads into the 2D window g[a] g[b] centred on it
    expect = np.zeros((15, 17))
    for a in range(11):
        for b in range(11):
            i, j = 3 + a - 5, 4 + b - 5
            if 0 <= i < 15 and 0 <= j < 17:
                expect[i, j] = g[a] * g[b]
    assert np.allclose(out, expect, rtol=0, atol=1e-17)


def test_ssim_of_an_image_with_itself_is_one_and_the_loss_vanishes():
    rng = np.random.default_rng(1)
    x = rng.random((20, 23, 3))
    assert abs(T.ssim(x, x) - 1.0) < 1e-14
    loss, grad = T.loss_l1_dssim(x, x)
    assert abs(loss) < 1e-14
    assert np.abs(grad).max() < 1e-12


def test_ssim_is_symmetric():
    rng = np.random.default_rng(2)
    x, y = rng.random((14, 9, 3)), rng.random((14, 9, 3))
    assert abs(T.ssim(x, y) - T.ssim(y, x)) < 1e-14


def test_single_pixel_closed_form():
    """A 1x1 image sees only the window's centre weight wc = g[5]^2 (zero
    padding): u = wc x, Sxx = wc x^2, Sxy = wc x y, so sigma_x^2 = wc (1 - wc) x^2
    and the map follows in closed form with C1 = 0.01^2, C2 = 0.03^2."""
    g = T.gaussian_window()
    wc = g[5] ** 2
    x, y = 0.7, 0.2
    u, v = wc * x, wc * y
    sx2, sy2, sxy = wc * (1 - wc) * x * x, wc * (1 - wc) * y * y, wc * (1 - wc) * x * y
    c1, c2 = 1e-4, 9e-4
    expect = (2 * u * v + c1) * (2 * sxy + c2) / ((u * u + v * v + c1) * (sx2 + sy2 + c2))
    got = T.ssim_terms(np.array([[x]]), np.array([[y]]))["map"][0, 0]
    assert np.isclose(got, expect, rtol=1e-14)


def test_constant_images_interior_closed_form():
    """Far from the border, constant images a and b have zero local variance,
    so the map is (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.8, 0.3
    s = T.ssim_terms(np.full((31, 33), a), np.full((31, 33), b))["map"]
    expect = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    assert np.allclose(s[5:-5, 5:-5], expect, rtol=1e-12)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    x = rng.random((9, 12, 3))
    y = rng.random((9, 12, 3))
    _, grad = T.loss_l1_dssim(x, y)
    h = 1e-6
    num = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        num[idx] = (T.loss_l1_dssim(xp, y)[0] - T.loss_l1_dssim(xm, y)[0]) / (2 * h)
    assert np.abs(num - grad).max() <= 1e-7 * np.abs(grad).max()


def test_l1_weight_and_view_mean():
    """With lam = 0 the loss is the mean absolute error; the multi-view loss is
    the mean of the views' losses."""
    rng = np.random.default_rng(4)
    x, y = rng.random((6, 7, 3)), rng.random((6, 7, 3))
    assert np.isclose(T.loss_l1_dssim(x, y, lam=0.0)[0], np.abs(x - y).mean(), rtol=1e-14)
    x2, y2 = rng.random((5, 4, 3)), rng.random((5, 4, 3))
    lv, gv = T.loss_views([x, x2], [y, y2])
    assert np.isclose(lv, 0.5 * (T.loss_l1_dssim(x, y)[0] + T.loss_l1_dssim(x2, y2)[0]), rtol=1e-14)
    assert np.allclose(gv[1], 0.5 * T.loss_l1_dssim(x2, y2)[1], rtol=1e-14)


@pytest.mark.parametrize("lr", [1e-3, 0.05])
def test_adam_matches_torch(lr):
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    p_t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p_t], lr=lr, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 5):
        g = rng.standard_normal(50)
        p_t.grad = torch.tensor(g)
        opt.step()
        p, m, v = T.adam_step(p, g, m, v, step, lr)
        assert np.allclose(p, p_t.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_is_a_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = T.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-10)
