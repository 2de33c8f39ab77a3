"""HIP kernel-agnostic MCMC step (Sec. 3.4) against its oracle: the draws,
copy counts and copied parameters bit-exact, the new opacities within 2 ulp
(FP64 -expm1(log1p(-o)/N) on both sides, libraries differ in the last bit),
and the positional noise.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import mcmc as MO
from paper_2501_18630_amd import scenes

pytestmark = pytest.mark.gpu
PARAMS = MO.PARAMS


def _gpu_relocate(s, tau, rand):
    import torch
    from paper_2501_18630_amd import renderer
    n, m = s["means"].shape[0], s["lobe_betas"].shape[1]
    params = renderer.to_device(s)
    mc = renderer.MCMC(n, m)
    r = torch.as_tensor(rand.astype(np.uint32).view(np.int32)).cuda()
    cnt = mc.relocate(params, tau, r)
    torch.cuda.synchronize()
    return {k: params[k].cpu().numpy() for k in PARAMS}, int(cnt.item())


@pytest.mark.parametrize("n,dead_frac,seed", [(1, 0.0, 1), (1000, 0.3, 2), (300_001, 0.05, 3)])
def test_relocation_matches_oracle(n, dead_frac, seed):
    rng = np.random.default_rng(seed)
    s = scenes.uniform_box_scene(n, [-1, -1, 2], [1, 1, 6], m=2, seed=seed)
    s["opacities"][rng.random(n) < dead_frac] = rng.uniform(0, 0.005, 1).astype(np.float32)
    rand = rng.integers(0, 2**32, n, dtype=np.uint64)
    got, moved = _gpu_relocate(s, 0.005, rand)
    ref, target, copies = MO.mcmc_relocate(s, 0.005, rand)
    assert moved == int((target >= 0).sum())
    for k in PARAMS:
        if k != "opacities":
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    ulp = np.spacing(ref["opacities"].astype(np.float32))
    assert np.all(np.abs(got["opacities"] - ref["opacities"]) <= 2 * ulp)


def test_relocation_edge_cases():
    rng = np.random.default_rng(4)
    s = scenes.uniform_box_scene(500, [-1, -1, 2], [1, 1, 6], m=2, seed=4)
    rand = rng.integers(0, 2**32, 500, dtype=np.uint64)
    # all dead: nothing to copy from, nothing moves
    s0 = {k: v.copy() for k, v in s.items()}
    s0["opacities"][:] = 0.0
    got, moved = _gpu_relocate(s0, 0.005, rand)
    assert moved == 0
    for k in PARAMS:
        np.testing.assert_array_equal(got[k], s0[k])
    # none dead: unchanged
    s1 = {k: v.copy() for k, v in s.items()}
    s1["opacities"][:] = 0.5
    got, moved = _gpu_relocate(s1, 0.005, rand)
    assert moved == 0
    for k in PARAMS:
        np.testing.assert_array_equal(got[k], s1[k])
    # one live primitive: every dead one copies it
    s2 = {k: v.copy() for k, v in s.items()}
    s2["opacities"][:] = 0.0
    s2["opacities"][123] = 0.3
    got, moved = _gpu_relocate(s2, 0.005, rand)
    assert moved == 499
    for k in PARAMS:
        if k != "opacities":
            assert np.all(got[k] == s2[k][123]), k
    ref, _, _ = MO.mcmc_relocate(s2, 0.005, rand)
    assert np.all(np.abs(got["opacities"] - ref["opacities"]) <= 2 * np.spacing(ref["opacities"]))


def test_noise_matches_oracle():
    import torch
    from paper_2501_18630_amd import renderer
    rng = np.random.default_rng(6)
    s = scenes.uniform_box_scene(20000, [-1, -1, 2], [1, 1, 6], m=2, seed=6)
    s["opacities"][:50] = 1.0
    s["opacities"][50:8000] = rng.uniform(0, 0.05, 7950).astype(np.float32)  # visible displacements
    z = rng.standard_normal((20000, 3)).astype(np.float32)
    params = renderer.to_device(s)
    mc = renderer.MCMC(20000, 2)
    mc.noise(params, torch.as_tensor(z).cuda(), 0.01, 5e4, float(np.log(25.0)))
    torch.cuda.synchronize()
    ref = MO.mcmc_noise(s, z, 0.01, 5e4, np.log(25.0))
    got = params["means"].cpu().numpy().astype(np.float64)
    d = ref - s["means"].astype(np.float64)        # the displacement itself to 1e-5
    np.testing.assert_allclose(got - s["means"], d, rtol=1e-4, atol=1e-5 * np.abs(d).max() + 1e-7)
    np.testing.assert_array_equal(params["means"].cpu().numpy()[:50], s["means"][:50])  # o = 1: no noise
