"""The loss of Eq. 7 for one pair of rendered views, and its gradient with
respect to both views, in numpy binary64.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
path. Shares no code with the GPU implementation.

Eq. 7 sums, over pairs (i, j), an L1 colour term, an SSIM term and an L1
depth term between the images rendered for i and j, weighted 0.8, 0.2 and
0.1 (Sec. 4.1). Readings, as for the separate terms:
  - |.|_1 is the mean absolute difference over the 3 W H colour values
    (and the W H depths), with sign(0) = 0 in its gradient;
  - the SSIM term is w_ssim (1 - mean SSIM) with the SSIM of oracle/ssim.py
    (11x11 Gaussian window, std 1.5, C1 = 0.01^2, C2 = 0.03^2, zero padding);
  - both rendered views depend on the parameters, so the gradient goes to
    both: SSIM(x, y) is symmetric in x and y, so its gradient with respect to
    the second image is the first-image gradient with the images swapped.
"""
import numpy as np

from . import ssim as S


def pair_loss_grad(rgb_i, rgb_j, depth_i, depth_j, w_l1=0.8, w_ssim=0.2, w_geom=0.1):
    """(loss, (g_rgb_i, g_rgb_j, g_depth_i, g_depth_j)) in binary64."""
    x, y = np.asarray(rgb_i, np.float64), np.asarray(rgb_j, np.float64)
    di, dj = np.asarray(depth_i, np.float64), np.asarray(depth_j, np.float64)
    n, p = x.size, di.size
    l1 = w_l1 * np.abs(x - y).sum() / n
    g1 = w_l1 * np.sign(x - y) / n
    ls, gxs = S.ssim_loss_grad(x, y, w_ssim)
    _, gys = S.ssim_loss_grad(y, x, w_ssim)
    ld = w_geom * np.abs(di - dj).sum() / p
    gd = w_geom * np.sign(di - dj) / p
    return l1 + ls + ld, (g1 + gxs, -g1 + gys, gd, -gd)
