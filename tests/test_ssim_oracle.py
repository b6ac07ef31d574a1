"""Pins of the SSIM oracle (oracle/ssim.py) against what the definition and
the mathematics fix, independently of its own code paths: the window sum
against a direct 2-D sum, closed forms of the SSIM map on constant and
checkerboard images (which pin C1, C2 and the window), the optimum x = y,
and the analytic gradient against central differences of the loss."""
import numpy as np

from oracle import ssim as S


def test_window_is_a_normalised_gaussian():
    g = S.window_1d()
    assert g.shape == (11,)
    assert abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    # neighbouring weights differ by the Gaussian ratio exp((2k + 1) / (2 sigma^2))
    for k in range(5):
        assert abs(g[5 - k] / g[4 - k] - np.exp((2 * k + 1) / (2 * 1.5 ** 2))) < 1e-12


def test_separable_blur_equals_the_direct_window_sum():
    rng = np.random.default_rng(3)
    img = rng.random((2, 9, 14))
    g = S.window_1d()
    w2 = np.outer(g, g)
    out = S.blur(img)
    for c, yq, xq in [(0, 0, 0), (1, 4, 7), (0, 8, 13), (1, 2, 12), (0, 6, 1)]:
        acc = 0.0
        for dy in range(-5, 6):
            for dx in range(-5, 6):
                yy, xx = yq + dy, xq + dx
                if 0 <= yy < 9 and 0 <= xx < 14:
                    acc += w2[dy + 5, dx + 5] * img[c, yy, xx]
        assert abs(out[c, yq, xq] - acc) < 1e-14, (c, yq, xq)


def test_constant_images_closed_form():
    # away from the border every statistic is exact: sigma terms vanish and
    # SSIM = (2 mx my + C1) / (mx^2 + my^2 + C1)
    mx, my = 0.7, 0.25
    x = np.full((1, 30, 30), mx)
    y = np.full((1, 30, 30), my)
    m = S.ssim_map(x, y)[0, 5:25, 5:25]
    want = (2 * mx * my + 0.01 ** 2) / (mx * mx + my * my + 0.01 ** 2)
    assert np.allclose(m, want, rtol=1e-12, atol=0)


def test_checkerboard_against_constant_closed_form():
    # x = m + a (-1)^(i+j), y = m: with s = sum_k g_k (-1)^k, at an interior
    # pixel of sign e the window gives mu_x = m + e a s^2, E[x^2] = m^2 + a^2 +
    # 2 m e a s^2, sigma_x^2 = a^2 (1 - s^4), sigma_xy = 0, hence
    # SSIM = (2 mu_x m + C1) C2 / ((mu_x^2 + m^2 + C1)(a^2 (1 - s^4) + C2))
    m, a = 0.5, 0.2
    i, j = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    sign = np.where((i + j) % 2 == 0, 1.0, -1.0)
    x = (m + a * sign)[None]
    y = np.full_like(x, m)
    s = sum(gk * (-1) ** k for k, gk in enumerate(S.window_1d()))
    got = S.ssim_map(x, y)[0]
    for (yq, xq) in [(10, 10), (10, 11), (16, 21), (21, 16)]:
        e = sign[yq, xq]
        mu = m + e * a * s * s
        want = (2 * mu * m + 0.01 ** 2) * 0.03 ** 2 / ((mu * mu + m * m + 0.01 ** 2) * (a * a * (1 - s ** 4) + 0.03 ** 2))
        assert abs(got[yq, xq] - want) < 1e-12 * abs(want), (yq, xq, got[yq, xq], want)


def test_identical_images_are_the_optimum():
    rng = np.random.default_rng(5)
    x = rng.random((3, 17, 12))
    loss, grad = S.ssim_loss_grad(x, x, 0.2)
    assert abs(loss) < 1e-14
    assert np.abs(grad).max() < 1e-15
    assert np.allclose(S.ssim_map(x, x), 1.0, rtol=0, atol=1e-14)


def test_gradient_against_central_differences():
    rng = np.random.default_rng(11)
    x = rng.random((2, 13, 16))
    y = np.clip(x + 0.3 * rng.standard_normal(x.shape), 0, 1)
    w = 0.2
    _, grad = S.ssim_loss_grad(x, y, w)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 6, 7), (0, 12, 15), (1, 0, 9), (0, 7, 0), (1, 12, 3)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (S.ssim_loss(xp, y, w) - S.ssim_loss(xm, y, w)) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(abs(fd), 1e-6), (idx, fd, grad[idx])
