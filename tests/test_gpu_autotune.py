"""The launch-shape autotuner on a small scene: it returns one of the
candidates it was given, times every candidate in the first round, re-times
the close ones in the finalist round, picks the fastest finalist, and a
cached choice is returned as it was stored."""
import numpy as np
import pytest
import torch

import synth
from paper_2602_23040_amd import autotune
from parity import atlas_tensor, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def test_autotune_sweep_finalists_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("PACKUV_TUNE_CACHE", str(tmp_path / "tune.json"))
    sc = synth.random_scene(side=16, sh_degree=1, views=3, width=96, height=64, seed=5)
    atlas = atlas_tensor(sc)
    cands = [(16, 16, 64), (8, 32, 64), (16, 16, 128)]
    t, info = autotune.choose(sc, atlas, candidates=cands, reps=2, final_reps=3, final_margin=10.0)
    say(f"[gpu] autotune: {info}")
    assert t in cands and info["source"] == "sweep"
    assert set(info["all_ms"]) == {"x".join(map(str, c)) for c in cands}
    assert all(np.isfinite(v) and v > 0 for v in info["all_ms"].values())
    # a margin that admits every candidate puts all three in the finalist round
    assert set(info["final_ms"]) == set(info["all_ms"])
    assert info["final_ms"]["x".join(map(str, t))] == min(info["final_ms"].values())
    t2, info2 = autotune.choose(sc, atlas, candidates=cands)
    assert t2 == t and info2["source"] == "cache"
