"""The batched step captured in a HIP graph: every replay, with eager work and
synchronisations between replays, reproduces the eager result bitwise
(images, loss and gradients)."""
import numpy as np
import pytest
import torch

import synth
from parity import atlas_tensor, renderer, run_forward, say

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = synth.random_scene(side=16, sh_degree=3, views=4, width=96, height=70, seed=8, lscale=(-2.9, 0.5))
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    tgt = torch.rand(3 * r.n_pixels, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(1))
    r.step(atlas, tgt)
    torch.cuda.synchronize()
    ref_img = r.image.clone()
    ref_g = r.dL_datlas.clone()
    ref_loss = float(r.loss.item())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.step(atlas, tgt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.step(atlas, tgt)
    torch.cuda.synchronize()
    for rep in range(4):
        say(f"[gpu] graph replay {rep}")
        # eager work between replays clobbers the buffers the graph writes
        r.image.fill_(-1.0)
        r.dL_datlas.fill_(7.0)
        r.sets[0].ranges.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.image, ref_img), f"replay {rep}: image differs"
        assert abs(float(r.loss.item()) - ref_loss) == 0.0
        assert torch.equal(r.dL_datlas, ref_g), f"replay {rep}: gradient differs"
    assert not r.overflowed()
    r.close()
