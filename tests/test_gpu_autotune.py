"""Launch-shape autotuner: picks a built shape, caches it per workload, and
the cached shape is returned without re-timing.  Needs an MI355X."""
import numpy as np
import pytest

from paper_2501_18630_amd import scenes

pytestmark = pytest.mark.gpu


def test_autotune_picks_and_caches(tmp_path):
    import torch
    from paper_2501_18630_amd import autotune, renderer
    s, cams = scenes.config0()
    params = renderer.to_device(s)
    target = torch.as_tensor(np.concatenate(
        [scenes.target_image(c["height"], c["width"], seed=1).reshape(-1) for c in cams])).cuda()
    cache = str(tmp_path / "tune.json")
    lines = []
    cfg = autotune.tune(cams, params, target, candidates=[(16, 16), (16, 8)], batches=[64, 128],
                        cache_path=cache, steps=2, refine=2, log=lines.append)
    assert (cfg.tile_w, cfg.tile_h) in [(16, 16), (16, 8)] and cfg.batch in (64, 128)
    assert sum(l.startswith("autotune refine") for l in lines) == 4
    again = autotune.tune(cams, params, target, cache_path=cache, log=lines.append)
    assert (again.tile_w, again.tile_h, again.batch) == (cfg.tile_w, cfg.tile_h, cfg.batch)
    assert sum(l.startswith("autotune") for l in lines) == 8  # nothing re-timed
