"""Pins of the oracle's compositing (Sec. 3.2, Eqs. 5-6) against closed
forms and invariants (CPU only)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2501_18630_amd import scenes

AMAX, TEPS = np.float64(np.float32(0.99)), np.float64(np.float32(1e-4))


def splats(rows, m=0):
    """rows: list of dicts(mu, s, q, o, b, c0)."""
    n = len(rows)
    return dict(means=np.array([r["mu"] for r in rows], np.float64),
                scales=np.array([r.get("s", (0.1, 0.1, 0.1)) for r in rows], np.float64),
                quats=np.array([r.get("q", (1, 0, 0, 0)) for r in rows], np.float64),
                opacities=np.array([r.get("o", 0.5) for r in rows], np.float64),
                betas=np.array([r.get("b", 0.0) for r in rows], np.float64),
                diffuse=np.array([r.get("c0", (1, 1, 1)) for r in rows], np.float64),
                lobe_angles=np.zeros((n, m, 2)), lobe_colors=np.zeros((n, m, 3)),
                lobe_betas=np.zeros((n, m)))


def image(out, cam):
    return out["rgb"].reshape(cam["height"], cam["width"], 3)


def test_single_isotropic_footprint_closed_form(oracle):
    # alpha(x) = o (1 - |x - c|^2 / R^2)^(4 e^b) inside the disc of radius R = f s / z, 0 outside
    W = H = 48
    f, z, s, o, b = 48.0, 3.0, 0.5, 0.7, 0.3
    cam = scenes.camera(W, H, f=f)
    out = oracle.render(splats([dict(mu=(0, 0, z), s=(s, s, s), o=o, b=b)]), cam, AMAX, 0.0)
    R = f * s / z
    yy, xx = np.mgrid[0:H, 0:W] + 0.5
    d2 = ((xx - W / 2) ** 2 + (yy - H / 2) ** 2) / R ** 2
    ref = np.where(d2 < 1, o * np.clip(1 - d2, 0, None) ** (4 * np.exp(b)), 0.0)
    np.testing.assert_allclose(image(out, cam)[..., 0], ref, atol=1e-13)
    # exactly the background outside the support, and T = 1 - alpha
    assert np.all(image(out, cam)[d2 >= 1] == 0.0)
    np.testing.assert_allclose(out["T"].reshape(H, W), 1 - ref, atol=1e-13)


def test_lit_pixels_are_the_centres_inside_the_rotated_ellipse(oracle):
    W, H, f, z = 64, 64, 64.0, 4.0
    sx, sy, th = 0.9, 0.3, 0.6
    cam = scenes.camera(W, H, f=f)
    q = (np.cos(th / 2), 0, 0, np.sin(th / 2))
    out = oracle.render(splats([dict(mu=(0.05, -0.1, z), s=(sx, sy, 0.2), q=q, o=0.9)]), cam, AMAX, 0.0)
    yy, xx = np.mgrid[0:H, 0:W] + 0.5
    dx, dy = xx - (f * 0.05 / z + 32), yy - (f * -0.1 / z + 32)
    c, s = np.cos(th), np.sin(th)
    u, v = c * dx + s * dy, -s * dx + c * dy          # coordinates along the ellipse axes
    inside = (u / (f * sx / z)) ** 2 + (v / (f * sy / z)) ** 2 < 1
    lit = out["T"].reshape(H, W) < 1
    assert inside.sum() > 100
    np.testing.assert_array_equal(lit, inside)


def test_two_splats_front_to_back_order(oracle):
    W = H = 16
    cam = scenes.camera(W, H, f=16.0, background=(0.2, 0.3, 0.4))
    front = dict(mu=(0, 0, 3.0), s=(1.0, 1.0, 1.0), o=0.6, b=0.0, c0=(1.0, 0.0, 0.0))
    back = dict(mu=(0, 0, 5.0), s=(2.0, 2.0, 2.0), o=0.5, b=0.5, c0=(0.0, 1.0, 0.0))
    pix = np.array([[8, 8], [3, 9]])
    for rows in ([front, back], [back, front]):      # input order must not matter
        out = oracle.render(splats(rows), cam, AMAX, 0.0, pixels=pix)
        for k, (u, v) in enumerate(pix):
            p = np.array([u + 0.5, v + 0.5]) - 8.0
            a1 = 0.6 * max(0, 1 - p @ p / (16 * 1.0 / 3) ** 2) ** 4
            a2 = 0.5 * max(0, 1 - p @ p / (16 * 2.0 / 5) ** 2) ** (4 * np.exp(0.5))
            ref = np.array([1, 0, 0]) * a1 + np.array([0, 1, 0]) * a2 * (1 - a1) \
                + np.array([0.2, 0.3, 0.4]) * (1 - a1) * (1 - a2)
            np.testing.assert_allclose(out["rgb"][k], ref, atol=1e-14)
            np.testing.assert_allclose(out["T"][k], (1 - a1) * (1 - a2), atol=1e-15)


def test_alpha_clamp(oracle):
    cam = scenes.camera(8, 8, f=8.0)
    # radius f s / z = 40 px; the pixel centre is 0.5 px off-centre in x and y
    out = oracle.render(splats([dict(mu=(0, 0, 2.0), s=(10, 10, 10), o=1.0)]), cam, AMAX, 0.0,
                        pixels=np.array([[4, 4], [4, 4]]))
    B = (1 - 0.5 / 40 ** 2) ** 4
    assert B > AMAX
    assert out["T"][0] == pytest.approx(1 - AMAX, abs=1e-15)
    out = oracle.render(splats([dict(mu=(0, 0, 2.0), s=(10, 10, 10), o=0.9)]), cam, AMAX, 0.0,
                        pixels=np.array([[4, 4]]))
    assert out["T"][0] == pytest.approx(1 - 0.9 * B, abs=1e-15)


def random_scene(n, seed, m=2, box=((-1, -1, 2), (1, 1, 5)), opaque=False):
    s = scenes.uniform_box_scene(n, box[0], box[1], m=m, seed=seed)
    s = {k: v.astype(np.float64) for k, v in s.items()}
    if opaque:
        s["opacities"] = np.full(n, 0.95)
        s["scales"] *= 3
    return s


def test_partition_of_unity(oracle):
    # colour = 1 and background = 1  =>  sum_i alpha_i T_i + T_final = 1 at every pixel
    s = random_scene(64, 11, m=2, opaque=True)
    s["diffuse"][:] = 1.0
    s["lobe_colors"][:] = 0.0
    cam = scenes.camera(32, 32, f=32.0, background=(1.0, 1.0, 1.0))
    for teps in (0.0, TEPS, 0.05):
        out = oracle.render(s, cam, AMAX, teps)
        np.testing.assert_allclose(out["rgb"], 1.0, atol=1e-13)


def test_early_termination_bound(oracle):
    s = random_scene(200, 12, m=2, opaque=True)
    cam = scenes.camera(32, 32, f=32.0, background=(0.3, 0.6, 0.9))
    full = oracle.render(s, cam, AMAX, 0.0)
    proj = oracle.project(s, cam)
    cmax = max(np.abs(proj["color"]).max(), 0.9)
    for teps in (TEPS, 0.01, 0.1):
        out = oracle.render(s, cam, AMAX, teps)
        assert np.all(np.abs(out["rgb"] - full["rgb"]) <= teps * cmax + 1e-14)
        stopped = out["T"] < teps
        assert np.all(out["T_prev"][stopped] >= teps)
    assert (oracle.render(s, cam, AMAX, 0.01)["T"] < 0.01).any()


def test_explicit_product_form_of_eq6(oracle):
    """C = sum_i c_i a_i prod_{j<i} (1 - a_j) + bg prod_j (1 - a_j), evaluated
    from the oracle's own projection with explicit products (no recursion)."""
    s = random_scene(40, 13, m=2)
    cam = scenes.camera(24, 20, f=24.0, background=(0.1, 0.2, 0.3))
    out = oracle.render(s, cam, AMAX, 0.0)
    p = oracle.project(s, cam)
    order = np.lexsort((np.arange(40), p["depth_key"]))
    order = order[p["valid"][order] == 1]
    k = 0
    for v in range(20):
        for u in range(24):
            d = np.array([u + 0.5, v + 0.5]) - p["mean2d"][order]
            A = p["conic"][order]
            r2 = A[:, 0] * d[:, 0] ** 2 + 2 * A[:, 1] * d[:, 0] * d[:, 1] + A[:, 2] * d[:, 1] ** 2
            a = np.where(r2 < 1, np.minimum(AMAX, s["opacities"][order]
                                            * np.clip(1 - r2, 0, None) ** p["beta"][order]), 0.0)
            ref = cam["background"].astype(np.float64) * np.prod(1 - a)
            for i in range(len(order)):
                ref = ref + p["color"][order[i]] * a[i] * np.prod(1 - a[:i])
            np.testing.assert_allclose(out["rgb"][k], ref, atol=1e-13)
            k += 1


def test_permutation_invariance(oracle):
    s = random_scene(80, 14, m=2)
    cam = scenes.camera(24, 24, f=24.0)
    ref = oracle.render(s, cam, AMAX, TEPS)
    perm = np.random.default_rng(0).permutation(80)
    out = oracle.render({k: v[perm] for k, v in s.items()}, cam, AMAX, TEPS)
    np.testing.assert_array_equal(out["rgb"], ref["rgb"])
    np.testing.assert_array_equal(perm[out["last"][out["last"] >= 0]], ref["last"][ref["last"] >= 0])


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def test_rigid_motion_invariance(oracle):
    s = random_scene(60, 15, m=2)
    cam = scenes.camera(24, 24, f=24.0, background=(0.1, 0.1, 0.1))
    ref = oracle.render(s, cam, AMAX, TEPS)
    rot = Rotation.from_rotvec([0.3, -1.1, 0.5])
    Q, d = rot.as_matrix(), np.array([1.5, -2.0, 0.7])
    qx, qy, qz, qw = rot.as_quat()
    t = dict(s)
    t["means"] = s["means"] @ Q.T + d
    t["quats"] = _qmul(np.array([qw, qx, qy, qz]), s["quats"])
    th, ph = s["lobe_angles"][..., 0], s["lobe_angles"][..., 1]
    dirs = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1) @ Q.T
    t["lobe_angles"] = np.stack([np.arccos(np.clip(dirs[..., 2], -1, 1)),
                                 np.arctan2(dirs[..., 1], dirs[..., 0])], -1)
    R2 = np.eye(3) @ Q.T
    cam2 = dict(cam)
    cam2["viewmat"] = np.concatenate([R2, (-R2 @ d)[:, None]], 1)
    out = oracle.render(t, cam2, AMAX, TEPS)
    np.testing.assert_allclose(out["rgb"], ref["rgb"], atol=1e-10)


def test_uniform_scale_invariance(oracle):
    s = random_scene(60, 16, m=2)
    cam = scenes.camera(24, 24, f=24.0, t=[0.2, -0.1, 0.5])
    ref = oracle.render(s, cam, AMAX, TEPS)
    k = 2.5
    t = dict(s)
    t["means"] = s["means"] * k
    t["scales"] = s["scales"] * k
    cam2 = dict(cam)
    cam2["viewmat"] = cam["viewmat"].astype(np.float64) * np.array([1, 1, 1, k])
    cam2["near"] = cam["near"] * k
    out = oracle.render(t, cam2, AMAX, TEPS)
    np.testing.assert_allclose(out["rgb"], ref["rgb"], atol=1e-10)
