"""SSIM loss term and its gradient, in binary64 numpy.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
CPU-baseline leg, never by the product path. Shares no code with the GPU
implementation.

What is computed. The mapping objective (Eq. 7) weights an SSIM term
between a rendered image and its reference; the SSIM itself is the formula
of the evaluation-metrics appendix, (2 mu_x mu_y + C1)(2 sigma_xy + C2) /
((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)). The paper does not say
over which neighbourhood the means, variances and covariance are taken.
Readings (each listed in the design notes):
  - local statistics under an 11x11 Gaussian window of standard deviation
    1.5 px, weights normalised to sum 1 (the window of the original SSIM
    definition); sigma_x^2 = E[x^2] - mu_x^2, sigma_xy = E[xy] - mu_x mu_y;
  - C1 = 0.01^2 and C2 = 0.03^2 for intensities on [0, 1];
  - zero padding: the window of a pixel near the border covers zeros
    outside the image, so the SSIM map has one value per pixel;
  - the loss term is weight * (1 - mean SSIM) over all channels and pixels.
    Eq. 7 writes the SSIM itself, which would reward dissimilarity when
    minimised; 1 - SSIM is the form that penalises it.

Gradient with respect to the rendered image x (the reference y is fixed):
with A1 = 2 mu_x mu_y + C1, A2 = 2 sigma_xy + C2, B1 = mu_x^2 + mu_y^2 + C1,
B2 = sigma_x^2 + sigma_y^2 + C2 and S = A1 A2 / (B1 B2),
  dS/dmu_x = S (2 mu_y / A1 - 2 mu_y / A2 - 2 mu_x / B1 + 2 mu_x / B2),
  dS/dE[x^2] = -S / B2,   dS/dE[xy] = 2 S / A2,
and each statistic at pixel q is a window sum over pixels p, so
  dL/dx(p) = sum_q w(q - p) (a(q) + 2 x(p) b(q) + y(p) c(q))
with a, b, c the three partials times dL/dS = -weight / (number of terms),
i.e. the zero-padded window sum of a, b and c (the window is symmetric).
"""
import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d() -> np.ndarray:
    """Normalised 1-D Gaussian weights; the 2-D window is their outer product."""
    r = np.arange(WINDOW, dtype=np.float64) - WINDOW // 2
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def blur(img: np.ndarray) -> np.ndarray:
    """Window sum at every pixel of the last two axes, zero outside the image
    (rows first, then columns: the 2-D window is separable)."""
    img = np.asarray(img, dtype=np.float64)
    g = window_1d()
    h = WINDOW // 2
    H, W = img.shape[-2:]
    pad = np.pad(img, [(0, 0)] * (img.ndim - 2) + [(h, h), (h, h)])
    rows = sum(g[k] * pad[..., :, k:k + W] for k in range(WINDOW))
    return sum(g[k] * rows[..., k:k + H, :] for k in range(WINDOW))


def _stats(x, y):
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    A1 = 2.0 * mx * my + C1
    A2 = 2.0 * sxy + C2
    B1 = mx * mx + my * my + C1
    B2 = sxx + syy + C2
    return mx, my, A1, A2, B1, B2


def ssim_map(x, y) -> np.ndarray:
    """Per-pixel SSIM of images x and y ([..., H, W])."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    _, _, A1, A2, B1, B2 = _stats(x, y)
    return (A1 * A2) / (B1 * B2)


def ssim_loss(x, y, weight: float = 1.0) -> float:
    """weight * (1 - mean SSIM) over every channel and pixel."""
    return float(weight * (1.0 - ssim_map(x, y).mean()))


def ssim_loss_grad(x, y, weight: float = 1.0):
    """(loss, dloss/dx) for x, y of shape [C, H, W]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx, my, A1, A2, B1, B2 = _stats(x, y)
    S = (A1 * A2) / (B1 * B2)
    dS = -weight / S.size
    a = dS * S * (2.0 * my / A1 - 2.0 * my / A2 - 2.0 * mx / B1 + 2.0 * mx / B2)
    b = dS * (-S / B2)
    c = dS * (2.0 * S / A2)
    grad = blur(a) + 2.0 * x * blur(b) + y * blur(c)
    return float(weight * (1.0 - S.mean())), grad
