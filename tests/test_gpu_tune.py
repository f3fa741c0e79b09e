"""Autotuner on the GPU: it measures every candidate launch shape on the
caller's workload, picks one, caches it, and the tuned launch renders the
same image as the default one."""
import json

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_forward

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_autotuner_measures_caches_and_keeps_images(tmp_path):
    from paper_2406_01579_amd import Params, SceneT
    from paper_2406_01579_amd.tune import Autotuner, candidates
    w = synth.training(s=320.0, R=24, size=128, views=2)
    sc = SceneT.from_numpy(w.scenes[0], "cuda")
    path = str(tmp_path / "tune.json")
    best = Autotuner(path, reps=2).best([sc], w.cams)
    cache = json.load(open(path))
    (key, entry), = cache.items()
    assert len(entry["ms"]) == len(candidates())
    assert all(v > 0 for v in entry["ms"].values())
    assert tuple(entry["best"]) == (best.tile_w, best.tile_h, best.waves, best.chunk_fwd, best.chunk_bwd)
    _, _, a = gpu_forward(w.scenes[0], w.cams, Params())
    _, _, b = gpu_forward(w.scenes[0], w.cams, best)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
