"""Pins of the FP64 loss oracle (Sec. 3.4 composite loss) against closed forms,
an independent separable evaluation and central finite differences."""
import numpy as np
import pytest

from oracle import loss as L


def _separable_mean(a, g):
    """Row then column 1D convolutions with zero padding ('same' size)."""
    r = g.size // 2
    rows = np.stack([np.convolve(np.pad(row, r), g[::-1], mode="valid") for row in a])
    return np.stack([np.convolve(np.pad(col, r), g[::-1], mode="valid") for col in rows.T]).T


def test_window_is_a_normalised_symmetric_gaussian():
    w = L.gaussian_window()
    assert w.shape == (11, 11)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    np.testing.assert_allclose(w, w[::-1, ::-1], rtol=0, atol=0)
    g = np.sqrt(np.diag(w))
    # g(k) / g(0) = exp(-k^2 / (2 sigma^2))
    np.testing.assert_allclose(g[5 + 2] / g[5], np.exp(-4 / (2 * 1.5 ** 2)), rtol=1e-13)


def test_window_mean_equals_separable_convolution():
    rng = np.random.default_rng(0)
    a = rng.uniform(0, 1, (17, 23))
    w = L.gaussian_window()
    g = np.sqrt(np.diag(w))
    np.testing.assert_allclose(L.window_mean(a, w), _separable_mean(a, g), rtol=1e-13, atol=1e-15)


def test_window_mean_adjoint_is_the_transpose():
    rng = np.random.default_rng(1)
    w = L.gaussian_window()
    a, d = rng.standard_normal((9, 14)), rng.standard_normal((9, 14))
    assert np.sum(L.window_mean(a, w) * d) == pytest.approx(np.sum(a * L.window_mean_adjoint(d, w)), rel=1e-12)


def test_ssim_of_identical_images_is_one_and_symmetric():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(0, 1, (15, 12)), rng.uniform(0, 1, (15, 12))
    np.testing.assert_allclose(L.ssim_map(x, x), 1.0, rtol=1e-12)
    np.testing.assert_allclose(L.ssim_map(x, y), L.ssim_map(y, x), rtol=1e-12)
    assert np.all(L.ssim_map(x, y) < 1.0)


def test_ssim_of_constant_images_interior():
    a, b = 0.3, 0.8
    s = L.ssim_map(np.full((20, 20), a), np.full((20, 20), b))
    expect = (2 * a * b + L.C1) / (a * a + b * b + L.C1)  # variances vanish: (C2 / C2)
    np.testing.assert_allclose(s[5:15, 5:15], expect, rtol=1e-12)


def test_ssim_constant_against_checkerboard_interior():
    """x = a, y = b + d (-1)^(i+j): with q = sum_k g_k (-1)^k the window gives
    mu_y = b + d (-1)^(i+j) q^2, var_y = d^2 (1 - q^4), cov = 0."""
    a, b, d = 0.4, 0.5, 0.2
    ii, jj = np.meshgrid(np.arange(24), np.arange(24), indexing="ij")
    sgn = (-1.0) ** (ii + jj)
    y = b + d * sgn
    g = np.sqrt(np.diag(L.gaussian_window()))
    q = np.sum(g * (-1.0) ** np.arange(-5, 6))
    mu_y = b + d * sgn * q * q
    var_y = d * d * (1 - q ** 4)
    expect = (2 * a * mu_y + L.C1) * L.C2 / ((a * a + mu_y * mu_y + L.C1) * (var_y + L.C2))
    s = L.ssim_map(np.full((24, 24), a), y)
    np.testing.assert_allclose(s[5:19, 5:19], expect[5:19, 5:19], rtol=1e-10)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_photometric_gradient_matches_central_differences(lam):
    rng = np.random.default_rng(3)
    x, y = rng.uniform(0, 1, (3, 9, 13)), rng.uniform(0, 1, (3, 9, 13))
    loss, g = L.photometric_loss(x, y, lam)
    h = 1e-6
    fd = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd[idx] = (L.photometric_loss(xp, y, lam)[0] - L.photometric_loss(xm, y, lam)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-9)


def test_photometric_loss_values():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (3, 8, 10))
    # identical images: no loss, and SSIM is at its maximum (zero gradient)
    l0, g0 = L.photometric_loss(x, x, 1.0)
    assert l0 == pytest.approx(0.0, abs=1e-14)
    np.testing.assert_allclose(g0, 0.0, atol=1e-12)
    # lam = 0: plain mean absolute error
    y = rng.uniform(0, 1, x.shape)
    l1, g1 = L.photometric_loss(x, y, 0.0)
    assert l1 == pytest.approx(np.abs(x - y).mean(), rel=1e-14)
    np.testing.assert_allclose(g1, np.sign(x - y) / x.size, rtol=0, atol=0)


def test_regularizer_closed_form():
    o = np.array([0.1, 0.0, 0.7])
    s = np.array([[0.1, 0.2, 0.3], [1.0, 2.0, 0.5], [0.01, 0.01, 0.01]])
    v, go, gs = L.regularizers(o, s, 0.01, 0.02)
    assert v == pytest.approx(0.01 * 0.8 + 0.02 * (0.6 + 3.5 + 0.03), rel=1e-14)
    np.testing.assert_array_equal(go, [0.01, 0.0, 0.01])
    np.testing.assert_array_equal(gs, np.full((3, 3), 0.02))
