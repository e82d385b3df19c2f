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


def test_graph_replays_with_adam_count_steps():
    """A captured step that ends with the Adam update: replays advance the
    device step counter, so k replays equal k eager steps bitwise (atlas,
    moments, counter)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = synth.random_scene(side=14, sh_degree=2, views=3, width=80, height=60, seed=9, lscale=(-2.9, 0.5))
    tgt = torch.rand(3 * sum(c.width * c.height for c in sc.cams), device="cuda:0",
                     generator=torch.Generator("cuda:0").manual_seed(2))
    # eager reference: three steps
    re = renderer(sc)
    a_eager = atlas_tensor(sc)
    run_forward(re, a_eager)
    re.grow_capacity(2.0, headroom=True)
    for _ in range(3):
        re.step(a_eager, tgt, adam=True)
    torch.cuda.synchronize()
    assert not re.overflowed()
    # captured: warm-up step on a side stream, capture, then two replays
    rg = renderer(sc)
    a_graph = atlas_tensor(sc)
    run_forward(rg, a_graph)
    rg.grow_capacity(2.0, headroom=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rg.step(a_graph, tgt, adam=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):        # capture records the step without running it
        rg.step(a_graph, tgt, adam=True)
    for rep in range(2):
        say(f"[gpu] adam graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
    assert not rg.overflowed()
    assert int(rg.adam_t.item()) == int(re.adam_t.item()) == 3
    assert torch.equal(rg.adam_m, re.adam_m) and torch.equal(rg.adam_v, re.adam_v)
    assert torch.equal(a_graph, a_eager)
    re.close()
    rg.close()


def test_captured_overflow_is_reported_then_recaptured():
    """A captured step with an instance capacity forced too small from the
    host: the replay overflows, check() (pg_status_check) reports it with the
    count that suffices, and after growing and capturing again every replay
    equals the eager step bitwise (images, loss, gradients)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = synth.random_scene(side=16, sh_degree=3, views=4, width=96, height=70, seed=8, lscale=(-2.9, 0.5))
    atlas = atlas_tensor(sc)
    tgt = torch.rand(3 * sc.n_pixels, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(3))
    re = renderer(sc)
    run_forward(re, atlas)
    re.step(atlas, tgt)
    torch.cuda.synchronize()
    ref = (re.image.clone(), re.dL_datlas.clone(), float(re.loss.item()))
    need_eager = int(re.sets[0].n_inst[0].item())
    re.close()

    r = renderer(sc, cap=64)
    r.check_overflow = False          # keep the tiny buffers for the capture
    stream = torch.cuda.current_stream()

    def capture():
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            r.step(atlas, tgt)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            r.step(atlas, tgt)
        torch.cuda.synchronize()
        return g

    g = capture()
    say("[gpu] replay with capacity 64")
    g.replay()
    torch.cuda.synchronize()
    [(ovf, need)] = r.status()
    assert ovf and need == need_eager > 64
    assert not r.check()
    assert r.ensure_capacity() and r.sets[0].cap >= need
    del g
    g = capture()
    for rep in range(3):
        say(f"[gpu] replay {rep} after re-capture")
        r.image.fill_(-1.0)
        r.dL_datlas.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert r.check()
        assert torch.equal(r.image, ref[0]) and torch.equal(r.dL_datlas, ref[1])
        assert float(r.loss.item()) == ref[2]
    r.close()
