"""FP64 reference of the training step around the renderer: the image loss
and the optimiser update.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

The paper trains with the rendering loss of 3D Gaussian Splatting, an l1 term
plus a D-SSIM term weighted 0.2 (Sec. 5, implementation details), and with the
EXP / LC weight parameters initialised as it states there.  The loss here is

    L = (1 - lam) * mean|x - y| + lam * (1 - mean SSIM(x, y)),   lam = 0.2,

with SSIM computed per colour channel as in Wang et al. (2004): local
statistics under an 11 x 11 Gaussian window of standard deviation 1.5 with
zero padding ("same" size), constants C1 = 0.01^2 and C2 = 0.03^2 (dynamic
range 1), and the mean taken over all pixels and channels.  For several views
the loss is the mean of the per-view losses.

The optimiser is Adam (Kingma and Ba, 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1D Gaussian taps g[k] ~ exp(-(k - c)^2 / (2 sigma^2)), c = size // 2."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def filter2(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out[i, j] = sum_{a, b} g[a] g[b] img[i + a - c, j + b - c], with img taken
    as zero outside its extent (the separable 2D Gaussian, same-size output)."""
    c = len(g) // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * c, W + 2 * c), dtype=np.float64)
    pad[c:c + H, c:c + W] = img
    rows = np.zeros((H + 2 * c, W), dtype=np.float64)
    for b in range(len(g)):
        rows += g[b] * pad[:, b:b + W]
    out = np.zeros((H, W), dtype=np.float64)
    for a in range(len(g)):
        out += g[a] * rows[a:a + H, :]
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray, g: np.ndarray | None = None) -> dict:
    """Per-pixel SSIM of two single-channel images and the partial derivatives
    of the map with respect to the windowed statistics u = G*x, Sxx = G*x^2
    and Sxy = G*(x y) (the statistics the map depends on through x)."""
    g = gaussian_window() if g is None else g
    u = filter2(x, g)
    v = filter2(y, g)
    sxx = filter2(x * x, g)
    syy = filter2(y * y, g)
    sxy = filter2(x * y, g)
    a1 = 2.0 * u * v + C1
    a2 = 2.0 * (sxy - u * v) + C2
    b1 = u * u + v * v + C1
    b2 = (sxx - u * u) + (syy - v * v) + C2
    s = a1 * a2 / (b1 * b2)
    # dS/du: a1 and a2 both depend on u (2v and -2v), b1 (2u) and b2 (-2u)
    d_u = (2.0 * v * a2 - 2.0 * v * a1) / (b1 * b2) - s * (2.0 * u / b1 - 2.0 * u / b2)
    d_sxx = -s / b2
    d_sxy = 2.0 * a1 / (b1 * b2)
    return {"map": s, "d_u": d_u, "d_sxx": d_sxx, "d_sxy": d_sxy}


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    """Mean SSIM of two [H][W][C] images over pixels and channels."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean([ssim_terms(x[..., ch], y[..., ch])["map"] for ch in range(x.shape[2])]))


def loss_l1_dssim(img: np.ndarray, target: np.ndarray, lam: float = 0.2):
    """Loss of one view and its gradient with respect to ``img`` ([H][W][C])."""
    x = np.asarray(img, dtype=np.float64)
    y = np.asarray(target, dtype=np.float64)
    H, W, Cn = x.shape
    P = H * W * Cn
    g = gaussian_window()
    l1 = np.abs(x - y).sum() / P
    grad = (1.0 - lam) * np.sign(x - y) / P
    s_sum = 0.0
    for ch in range(Cn):
        t = ssim_terms(x[..., ch], y[..., ch], g)
        s_sum += t["map"].sum()
        # adjoint of the windowed statistics: the same (symmetric) filter
        dmean = (filter2(t["d_u"], g) + 2.0 * x[..., ch] * filter2(t["d_sxx"], g)
                 + y[..., ch] * filter2(t["d_sxy"], g)) / P
        grad[..., ch] -= lam * dmean
    loss = (1.0 - lam) * l1 + lam * (1.0 - s_sum / P)
    return loss, grad


def loss_views(imgs: list, targets: list, lam: float = 0.2):
    """Mean over views of the per-view loss; gradients per view."""
    out = [loss_l1_dssim(a, b, lam) for a, b in zip(imgs, targets)]
    V = len(out)
    return sum(o[0] for o in out) / V, [o[1] / V for o in out]


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam update (step counts from 1).  Returns new (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
