"""Reference of the kernel-agnostic MCMC step of Sec. 3.4: positional noise
(Optimization paragraph) and distribution-preserving relocation of dead
primitives (Densification paragraph and its appendix proof).

TEST INFRASTRUCTURE ONLY: used by tests/ and nothing else; it shares no code
with the HIP path and imports nothing from the product package.

Readings (the paper states the update, not these details):
  * noise: eps = lr B(o; b') eta with B(o; b') = (1 - o)^(4 e^b') the Beta
    kernel (b' = ln 25 gives (1 - o)^100), eta a sample of N(0, Sigma) for the
    primitive's covariance, eta = R diag(s) z with z ~ N(0, I) supplied by the
    caller; mu <- mu + lambda_eps eps.
  * relocation: a primitive is dead when o <= tau.  Each dead primitive i
    draws a live one j with probability proportional to its opacity, from
    the caller's uniform 32-bit integer u_i.  To make that draw an exact
    integer decision, opacities are weighed in units of 2^-24,
    w_j = floor(o_j 2^24), and i takes the j whose cumulative weight interval
    contains t_i = floor(u_i W / 2^32), W = sum_j w_j.  A live primitive
    chosen by N - 1 dead ones ends with N copies, all with opacity
    o' = 1 - (1 - o)^(1/N) (scales unchanged: only the opacity is adjusted).
"""
from __future__ import annotations

import numpy as np

QUANT = 1 << 24
PARAMS = ("means", "scales", "quats", "opacities", "betas", "diffuse",
          "lobe_angles", "lobe_colors", "lobe_betas")


def beta_kernel(x, b):
    """B(x; b) = (1 - x)^(4 e^b) (Sec. 3.1)."""
    return (1.0 - np.asarray(x, np.float64)) ** (4.0 * np.exp(b))


def rotation(q):
    """R of the normalised quaternion (w, x, y, z), one per row."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def mcmc_noise(scene: dict, z: np.ndarray, lr: float, lam_eps: float, b_prime: float) -> np.ndarray:
    """New means: mu + lam_eps lr B(o; b') R diag(s) z."""
    mu = np.asarray(scene["means"], np.float64)
    s = np.asarray(scene["scales"], np.float64)
    eta = np.einsum("nij,nj->ni", rotation(scene["quats"]), s * np.asarray(z, np.float64))
    scale = lam_eps * lr * beta_kernel(scene["opacities"], b_prime)
    return mu + scale[:, None] * eta


def sample_targets(opacities: np.ndarray, tau: float, rand: np.ndarray):
    """Dead mask and, for every dead primitive, the live primitive it copies
    (-1 where there is none to copy)."""
    o = np.asarray(opacities, np.float32)
    dead = o <= np.float32(tau)
    w = np.where(dead, 0, np.floor(o.astype(np.float64) * QUANT)).astype(np.int64)
    total = int(w.sum())
    target = np.full(o.shape[0], -1, np.int64)
    if total == 0:
        return dead, target
    cum = np.cumsum(w)  # inclusive
    hi, lo = total >> 32, total & 0xFFFFFFFF
    for i in np.nonzero(dead)[0]:
        u = int(rand[i])
        t = u * hi + ((u * lo) >> 32)  # floor(u W / 2^32), exact
        target[i] = int(np.searchsorted(cum, t, side="right"))
    return dead, target


def mcmc_relocate(scene: dict, tau: float, rand: np.ndarray):
    """Returns (new scene dict of float32 arrays, target indices, copies per
    primitive)."""
    dead, target = sample_targets(scene["opacities"], tau, rand)
    n = dead.shape[0]
    copies = np.ones(n, np.int64)
    for j in target[target >= 0]:
        copies[j] += 1
    out = {k: np.array(scene[k], copy=True) for k in PARAMS}
    o = np.asarray(scene["opacities"], np.float64)
    chosen = copies > 1
    o_new = -np.expm1(np.log1p(-o[chosen]) / copies[chosen])  # 1 - (1 - o)^(1/N)
    out["opacities"][chosen] = o_new.astype(np.float32)
    for i in np.nonzero(target >= 0)[0]:
        j = target[i]
        for k in PARAMS:
            out[k][i] = out[k][j]
    return out, target, copies
