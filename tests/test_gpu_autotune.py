"""Autotuner on the GPU: it returns runnable options, caches them, and the
tuned batch gives the same dose as the default one (the options never change
which histories run)."""
import numpy as np
import pytest

from paper_0910_0329_amd import autotune
from paper_0910_0329_amd.inputs import configs, sources

pytestmark = pytest.mark.gpu


def test_tune_and_reuse(blob, tmp_path):
    import torch
    from paper_0910_0329_amd.mcdose import Engine
    assert torch.cuda.is_available()
    eng = Engine(0)
    try:
        th = eng.load_materials(blob)
        w = configs.photon_6mv_wbw(1)
        pid = eng.load_phantom(w.phantom, th)
        srcs, ns = sources.beamlets(w.phantom, seed=4)
        items = [(s, int(n) // 50 + 100, i) for i, (s, n) in enumerate(zip(srcs[:16], ns[:16]))]
        path = str(tmp_path / "tune.json")
        space = {"regroup": (1, 2, 3), "chunk_per_lane": (16, 64), "block_size": (256, 512),
                 "table_placement": (1, 2)}
        sched = {"sched_fetch_div": (3, 4), "sched_hard_div": (16,), "sched_photon_div": (4,)}
        opts = autotune.tune(eng, pid, w.phantom.n_vox, items, 4, space=space, sched_space=sched, scale=1,
                             reps=1, path=path, log=print)
        launch = {k: v for k, v in opts.items() if not k.startswith("sched_") and k != "grid_blocks"}
        assert launch in list(autotune.candidates(space))
        if "grid_blocks" in opts:
            shape = eng.launch_shape(pid, **launch)
            assert {"grid_blocks": opts["grid_blocks"]} in autotune.occupancy_candidates(shape)
        table = autotune.load_cache(path)
        tried = [t["opts"] for e in table.values() for t in e["table"]]
        # every stage-1 candidate ran, and the occupancy stage ran when the winner had one
        assert len(tried) >= len(list(autotune.candidates(space))) + len(sched["sched_fetch_div"])
        assert autotune.load_cache(path)
        again = autotune.tune(eng, pid, w.phantom.n_vox, items, 4, space=space, path=path)
        assert again == opts
        a, _ = eng.simulate_batch(pid, items, 4, n_vox=w.phantom.n_vox, **opts)
        b, _ = eng.simulate_batch(pid, items, 4, n_vox=w.phantom.n_vox)
        for x, y in zip(a, b):
            d0 = y["dose"].cpu().numpy()
            np.testing.assert_allclose(x["dose"].cpu().numpy(), d0, rtol=0, atol=1e-9 * d0.max())
    finally:
        eng.close()
