"""Pins of the MCMC oracle (Sec. 3.4): the distribution-preservation identity,
the weighted draw against an explicit lookup table, copy bookkeeping, and
closed forms of the positional noise."""
import numpy as np
import pytest

from oracle import mcmc as M


def _scene(n, rng, m=2):
    q = rng.standard_normal((n, 4))
    return dict(means=rng.uniform(-1, 1, (n, 3)).astype(np.float32),
                scales=np.exp(rng.uniform(-4, -1, (n, 3))).astype(np.float32),
                quats=(q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32),
                opacities=rng.uniform(0, 0.3, n).astype(np.float32),
                betas=rng.normal(0, 0.5, n).astype(np.float32),
                diffuse=rng.uniform(0, 1, (n, 3)).astype(np.float32),
                lobe_angles=rng.uniform(0, 3, (n, m, 2)).astype(np.float32),
                lobe_colors=rng.uniform(0, 0.5, (n, m, 3)).astype(np.float32),
                lobe_betas=rng.normal(0, 0.5, (n, m)).astype(np.float32))


def test_relocated_opacity_preserves_the_centre_alpha():
    """N copies of opacity o' composite to the original o at the kernel
    centre: 1 - (1 - o')^N = o (appendix, densification identity)."""
    rng = np.random.default_rng(0)
    s = _scene(400, rng)
    s["opacities"][:150] = 0.001
    out, target, copies = M.mcmc_relocate(s, 0.005, rng.integers(0, 2**32, 400, dtype=np.uint64))
    chosen = np.nonzero(copies > 1)[0]
    assert chosen.size > 20
    o = s["opacities"][chosen].astype(np.float64)
    o2 = out["opacities"][chosen].astype(np.float64)
    np.testing.assert_allclose(1 - (1 - o2) ** copies[chosen], o, rtol=2e-6)
    # and the small-opacity approximation o' ~ o / N of Sec. 3.4 holds to first order
    assert np.all(np.abs(o2 - o / copies[chosen]) <= o * o)


def test_draw_matches_an_explicit_table():
    """Opacities that are small multiples of 2^-24: the cumulative-weight
    search must agree with a table listing live j w_j times."""
    k = np.array([0, 3, 0, 5, 1, 0, 7, 2], np.int64)  # weights; zeros are dead (tau = 0)
    o = (k / M.QUANT).astype(np.float32)
    table = np.repeat(np.arange(k.size), k)
    rng = np.random.default_rng(1)
    rand = rng.integers(0, 2**32, k.size, dtype=np.uint64)
    dead, target = M.sample_targets(o, 0.0, rand)
    for i in np.nonzero(dead)[0]:
        t = (int(rand[i]) * int(k.sum())) >> 32
        assert target[i] == table[t]
    assert np.all(target[~dead] == -1)


def test_draw_frequencies_follow_opacity():
    n = 20000
    rng = np.random.default_rng(2)
    o = np.zeros(n, np.float32)
    o[:4] = [0.1, 0.2, 0.3, 0.4]
    dead, target = M.sample_targets(o, 0.005, rng.integers(0, 2**32, n, dtype=np.uint64))
    freq = np.bincount(target[dead], minlength=4)[:4] / dead.sum()
    np.testing.assert_allclose(freq, [0.1, 0.2, 0.3, 0.4], atol=0.01)


def test_copies_and_untouched_primitives():
    rng = np.random.default_rng(3)
    s = _scene(300, rng)
    s["opacities"][rng.random(300) < 0.3] = 0.0
    out, target, copies = M.mcmc_relocate(s, 0.005, rng.integers(0, 2**32, 300, dtype=np.uint64))
    dead = s["opacities"] <= 0.005
    assert np.array_equal(target >= 0, dead)
    assert copies.sum() - copies.size == dead.sum()
    for i in np.nonzero(dead)[0]:
        for key in M.PARAMS:
            np.testing.assert_array_equal(out[key][i], out[key][target[i]])
    keep = ~dead & (copies == 1)
    for key in M.PARAMS:
        np.testing.assert_array_equal(out[key][keep], s[key][keep])
    for key in M.PARAMS:
        if key != "opacities":
            np.testing.assert_array_equal(out[key][~dead], s[key][~dead])


def test_nothing_to_copy_from():
    s = _scene(10, np.random.default_rng(4))
    s["opacities"][:] = 0.0
    out, target, copies = M.mcmc_relocate(s, 0.005, np.arange(10, dtype=np.uint64))
    assert np.all(target == -1) and np.all(copies == 1)
    for key in M.PARAMS:
        np.testing.assert_array_equal(out[key], s[key])


def test_noise_closed_forms():
    rng = np.random.default_rng(5)
    s = _scene(4, rng)
    s["quats"][:] = [1, 0, 0, 0]                       # R = I
    s["quats"][3] = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]  # 90 degrees about z
    z = rng.standard_normal((4, 3)).astype(np.float32)
    lr, lam, bp = 0.3, 2.0, np.log(25.0)
    new = M.mcmc_noise(s, z, lr, lam, bp)
    o = s["opacities"].astype(np.float64)
    sc = s["scales"].astype(np.float64)
    amp = lam * lr * (1 - o) ** 100.0                 # 4 e^(ln 25) = 100
    np.testing.assert_allclose(new[:3], s["means"][:3] + amp[:3, None] * sc[:3] * z[:3], rtol=1e-12)
    eta3 = np.array([-sc[3, 1] * z[3, 1], sc[3, 0] * z[3, 0], sc[3, 2] * z[3, 2]])
    np.testing.assert_allclose(new[3], s["means"][3] + amp[3] * eta3, rtol=1e-6, atol=1e-12)
    assert M.beta_kernel(0.01, np.log(25.0)) == pytest.approx(0.99 ** 100, rel=1e-12)
