"""FP64 reference of the training loss of Sec. 3.4 (Optimization): the
photometric term (1 - lambda) L1 + lambda (1 - SSIM) of the composite loss
equation, and its two regularisers lambda_o sum_i |o_i| and
lambda_Sigma sum_i sum_j |sqrt(eig_j(Sigma_i))|.

TEST INFRASTRUCTURE ONLY: used by tests/ and nothing else; it shares no code
with the HIP path and imports nothing from the product package.

The paper names SSIM but not its window or constants; this follows the
standard definition (Wang et al. 2004) as 3D Gaussian Splatting trains with
it: an 11 x 11 Gaussian window with sigma 1.5, C1 = 0.01^2, C2 = 0.03^2 for
images in [0, 1], statistics taken per colour channel over the window with
zero padding outside the image (an output the size of the input), and the
loss averaged over all channel-pixels.  Views of a batch add their losses.

Everything is written out from the definition: the window statistics are
direct sums over the 121 window offsets (not separable passes), and the
gradient is the chain rule of those sums, one step at a time.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """2D window w(a, b) = g(a) g(b), g the normalised sampled Gaussian."""
    r = size // 2
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def window_mean(a: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_{a,b} w(a,b) img(y + a - r, x + b - r), zero outside the image."""
    r = w.shape[0] // 2
    h, wd = a.shape
    pad = np.zeros((h + 2 * r, wd + 2 * r))
    pad[r:r + h, r:r + wd] = a
    out = np.zeros((h, wd))
    for i in range(w.shape[0]):
        for j in range(w.shape[1]):
            out += w[i, j] * pad[i:i + h, j:j + wd]
    return out


def window_mean_adjoint(d: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of window_mean: img(q) receives w(a,b) d(p) for every p whose
    window reaches q (p = q - offset), zero-padded outputs contribute nothing."""
    r = w.shape[0] // 2
    h, wd = d.shape
    out = np.zeros((h + 2 * r, wd + 2 * r))
    for i in range(w.shape[0]):
        for j in range(w.shape[1]):
            out[i:i + h, j:j + wd] += w[i, j] * d
    return out[r:r + h, r:r + wd]


def ssim_map(x: np.ndarray, y: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
    for one channel; s_x^2 = E[x^2] - mu_x^2, s_xy = E[xy] - mu_x mu_y."""
    w = gaussian_window() if w is None else w
    mx, my = window_mean(x, w), window_mean(y, w)
    exx, eyy, exy = window_mean(x * x, w), window_mean(y * y, w), window_mean(x * y, w)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def photometric_loss(x: np.ndarray, y: np.ndarray, lam: float):
    """One view, x and y [3, H, W]: L = (1 - lam) mean|x - y| + lam (1 - mean SSIM).
    Returns (L, dL/dx)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = gaussian_window()
    n = x.size
    loss = (1.0 - lam) * np.abs(x - y).sum() / n + lam
    grad = (1.0 - lam) * np.sign(x - y) / n
    for c in range(x.shape[0]):
        xc, yc = x[c], y[c]
        mx, my = window_mean(xc, w), window_mean(yc, w)
        exx, eyy, exy = window_mean(xc * xc, w), window_mean(yc * yc, w), window_mean(xc * yc, w)
        a1 = 2 * mx * my + C1
        a2 = 2 * (exy - mx * my) + C2
        b1 = mx * mx + my * my + C1
        b2 = (exx - mx * mx) + (eyy - my * my) + C2
        s = a1 * a2 / (b1 * b2)
        loss -= lam * s.sum() / n
        # d s / d(mx, exx, exy), then through the window means back to x
        ds_dmx = (2 * my * a2 + a1 * (-2 * my)) / (b1 * b2) - s * (2 * mx / b1 - 2 * mx / b2)
        ds_dexx = -s / b2
        ds_dexy = 2 * a1 / (b1 * b2)
        gx = (window_mean_adjoint(ds_dmx, w) + 2 * xc * window_mean_adjoint(ds_dexx, w)
              + yc * window_mean_adjoint(ds_dexy, w))
        grad[c] -= lam * gx / n
    return loss, grad


def batch_photometric_loss(images, targets, lam: float):
    """Sum over views of photometric_loss; returns (L, [dL/dx per view])."""
    total, grads = 0.0, []
    for x, y in zip(images, targets):
        l, g = photometric_loss(x, y, lam)
        total += l
        grads.append(g)
    return total, grads


def regularizers(opacities: np.ndarray, scales: np.ndarray, lam_o: float, lam_s: float):
    """lam_o sum_i |o_i| + lam_s sum_i sum_j |sqrt(eig_j(Sigma_i))|.  With
    Sigma = R diag(s^2) R^T the eigenvalues are s_j^2, so the second sum is
    sum |s_j|.  Returns (value, dL/do, dL/ds)."""
    o = np.asarray(opacities, np.float64)
    s = np.asarray(scales, np.float64)
    val = lam_o * np.abs(o).sum() + lam_s * np.abs(s).sum()
    return val, lam_o * np.sign(o), lam_s * np.sign(s)
