"""The tile dispatch order that pg_bin_sort writes for the compositing calls:
every tile exactly once, longest list classes first, each class's tiles in
index order dealt to the XCDs in contiguous runs (checked slot by slot), and
the forward and the adjoint give bitwise the same images, entries and
gradient slots with it as with the default order (it schedules work,
nothing else)."""
import numpy as np
import pytest
import torch

import synth
from paper_2602_23040_amd import _abi as abi
from parity import atlas_tensor, renderer, run_forward, say

pytestmark = pytest.mark.gpu

SCENES = {
    "tiny": lambda: synth.random_scene(side=12, sh_degree=1, views=2, width=64, height=48, seed=0),
    "config2": lambda: synth.make_scene(2),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def length_class(n):
    """64 classes, four per octave of n + 1 (linear quarters), longest first."""
    x = n.astype(np.int64) + 1
    e = np.floor(np.log2(x)).astype(np.int64)
    e = np.where((1 << (e + 1)) <= x, e + 1, e)          # guard the floor of log2 at exact powers
    e = np.where((1 << e) > x, e - 1, e)
    q = ((x - (1 << e)) * 4) >> e                         # quarter of the octave
    return 63 - np.minimum(4 * e + q, 63)


def expected_order(lengths):
    """Classes longest first; inside a class, the tiles in index order dealt
    to the XCDs (slot mod 8) in contiguous runs."""
    cls = length_class(lengths)
    tiles = np.lexsort((np.arange(len(lengths)), cls))
    out = np.empty(len(lengths), np.int64)
    o = 0
    for c in range(64):
        run = tiles[o:o + int((cls == c).sum())]
        slots = np.arange(o, o + len(run))
        r = 0
        for x in range(8):
            sx = slots[slots % 8 == x]
            out[sx] = run[r:r + len(sx)]
            r += len(sx)
        o += len(run)
    return out


@pytest.mark.parametrize("name", list(SCENES))
def test_order_is_a_longest_first_permutation_and_changes_nothing(name):
    sc = SCENES[name]()
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    r.loss_l1(torch.rand(3 * r.n_pixels, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(3)))
    r.backward()
    torch.cuda.synchronize()
    s = r.sets[0]
    nt = s.info.n_tiles
    order = s.order[:nt].cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(nt)), "not a permutation of the tiles"
    rg = s.ranges[:2 * nt].cpu().numpy().reshape(nt, 2)
    cls = length_class(rg[order, 1] - rg[order, 0])
    assert np.all(np.diff(cls) >= 0), "list length classes are not in descending order"
    assert np.array_equal(order, expected_order(rg[:, 1] - rg[:, 0])), "order differs from the rule"
    say(f"[gpu] tile order {name}: {nt} tiles, longest list {int((rg[:, 1] - rg[:, 0]).max())} first")
    image, T, nc = r.image.clone(), r.final_T.clone(), r.n_contrib.clone()
    te, ent, slots = s.tile_entries.clone(), s.entries.clone(), s.inst_grad.clone()
    n_inst = int(s.n_inst[0].item())
    # the same calls in the default (neighbouring tiles together) order
    r.image.zero_()
    s.inst_grad.zero_()
    abi.pg_render_fwd(s.handle, s.splats, s.values, s.ranges, None, r.bg, r.image, r.final_T, r.n_contrib,
                      s.tile_entries, s.entries)
    abi.pg_render_bwd(s.handle, s.splats, s.tiles, s.values, s.ranges, None, s.inst_first, s.n_inst, s.cap,
                      s.tile_entries, s.entries, r.n_contrib, r.bg, r.final_T, r.dL_dimage, s.inst_grad)
    torch.cuda.synchronize()
    assert torch.equal(image, r.image) and torch.equal(T, r.final_T) and torch.equal(nc, r.n_contrib)
    assert torch.equal(te, s.tile_entries)
    assert torch.equal(ent[:n_inst], s.entries[:n_inst])
    assert torch.equal(slots[:abi.SLOT_WORDS * n_inst], s.inst_grad[:abi.SLOT_WORDS * n_inst])
    r.close()
