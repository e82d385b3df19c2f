"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded scenes (tiny ragged scenes, a multi-frame window, large
Gaussians whose rectangles exceed 64 tiles, Gaussians all at one depth, and the two
workloads small enough for the oracle to finish in seconds: the 64x64-atlas
single view and the 256x256-atlas ring of eight 512x512 views)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import (IMG_TOL, atlas_tensor, check_records, check_tile_lists, explain, gpu_images, gpu_n_contrib,
                    grad_compare, renderer, run_forward, say)

pytestmark = pytest.mark.gpu

SCENES = {
    "tiny": lambda: synth.random_scene(side=12, sh_degree=1, views=3, width=72, height=56, seed=0,
                                       lscale=(-2.8, 0.5)),
    "ragged": lambda: synth.random_scene(side=20, sh_degree=3, views=2, width=100, height=37, seed=1,
                                         occupancy=0.7, lscale=(-3.0, 0.6)),
    "multiframe": lambda: synth.random_scene(side=10, sh_degree=2, views=2, width=64, height=50, seed=2, frames=3,
                                             lscale=(-2.7, 0.5), dynamic_frac=0.5),
    # large Gaussians: rectangles of up to 110 tiles (more than 64 keep every tile)
    "large": lambda: synth.random_scene(side=8, sh_degree=1, views=2, width=200, height=150, seed=5,
                                        lscale=(-1.3, 0.4)),
    # every Gaussian at one depth in front of one camera: each pass of the depth sort sees a
    # single digit (the copy path) and the tile lists keep equal depths in id order
    "flat": lambda: synth.random_scene(side=12, sh_degree=1, views=0, width=64, height=48, seed=7,
                                       pos=((-1, -1, 3), (1, 1, 3)), lscale=(-3.4, 0.4)),
    # mostly opaque Gaussians (logit-opacity N(6, 1.5): about 80 % at o >= 0.99, with a few
    # dozen clamped pixels per view): the compositing kernels' clamped-alpha paths, and
    # pixels that stop early
    "opaque": lambda: synth.random_scene(side=14, sh_degree=1, views=2, width=80, height=60, seed=11,
                                         lscale=(-2.2, 0.4), lopac=(6.0, 1.5)),
    "config1": lambda: synth.make_scene(1),
    "config2": lambda: synth.make_scene(2),
}

_cache = {}


def case(name):
    if name not in _cache:
        say(f"[case] {name}: building scene and oracle forward")
        sc = SCENES[name]()
        fw = oracle.Forward(sc)
        _cache[name] = (sc, fw)
    return _cache[name]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


@pytest.mark.parametrize("name", list(SCENES))
def test_fetch_project_sort_bit_exact(name):
    sc, fw = case(name)
    say(f"[gpu] fetch/project/sort {name}")
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    N = r.N
    assert int(r.n_gauss_dev.item()) == N == fw.n_gauss
    assert np.array_equal(r.gauss_texel[:N].cpu().numpy(), fw.ids)
    tg = r.texel_gauss.cpu().numpy()
    exp_tg = np.full(sc.H * sc.W, -1, np.int32)
    exp_tg[fw.ids] = np.arange(N, dtype=np.int32)
    assert np.array_equal(tg, exp_tg)
    P = r.params[:sc.frames * sc.C * N].cpu().numpy().reshape(sc.frames, sc.C, N)
    assert np.array_equal(P.astype(np.float64), fw.params)
    spl, bins = r.splat_records(), r.bin_records()
    tsets = r.tile_sets()
    keys, vals = r.sorted_instances()
    tb = r.sets[0].tile_base
    ranges = r.sets[0].ranges.cpu().numpy().reshape(-1, 2).astype(np.int64)
    n_kept = 0
    for v in range(len(sc.cams)):
        pr = fw.proj[v]
        valid, listed = check_records(fw, v, bins, tsets, spl, N)
        s = spl[v * N:(v + 1) * N]
        np.testing.assert_allclose(s["conic"][valid], pr["conic"][valid], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(s["opacity"][valid], pr["opacity"][valid], rtol=1e-6)
        np.testing.assert_allclose(s["color"][valid], pr["color"][valid], rtol=1e-6, atol=1e-7)
        assert np.array_equal(s["depth"][valid].view(np.uint32), pr["key"][valid])
        kept = check_tile_lists(fw, v, keys, vals, tb, N)
        inst = fw.inst[v]
        # the kept count of each record is the number of its tiles left in the lists
        per_rec = np.bincount(inst["id"][kept], minlength=N)
        assert np.array_equal(per_rec, bins[v * N:(v + 1) * N]["n_tiles"].astype(np.int64))
        # ranges: each tile's [start, end) holds exactly its kept entries, tiles in order
        TX, TY = oracle.tiles_of(sc.cams[v], fw.tw, fw.th)
        per_tile = np.bincount(inst["tile"][kept], minlength=TX * TY)
        rg = ranges[tb[v]:tb[v + 1]]
        assert np.array_equal(rg[:, 1] - rg[:, 0], per_tile)
        nz = per_tile > 0
        assert np.array_equal(rg[nz, 0], n_kept + np.concatenate([[0], np.cumsum(per_tile)[:-1]])[nz])
        n_kept += int(kept.sum())
    assert keys.size == n_kept
    vis = r.visible[:sc.frames * N].cpu().numpy().reshape(sc.frames, N)
    assert np.array_equal(vis, fw.visible())
    r.close()


@pytest.mark.parametrize("name", list(SCENES))
def test_render_forward_parity(name):
    sc, fw = case(name)
    say(f"[gpu] render_fwd {name}")
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    imgs = gpu_images(r)
    keys, vals = r.sorted_instances()
    total_bad = total_unexp = 0
    for v in range(len(sc.cams)):
        gi, gT, gn = imgs[v]
        kept = check_tile_lists(fw, v, keys, vals, r.sets[0].tile_base, r.N)
        flips, unexp, nbad = explain(fw, v, gi, gT, gn, kept)
        total_bad += nbad
        total_unexp += len(unexp)
        ok = np.ones(gn.shape, bool)
        for p in flips:
            ok.reshape(-1)[p] = False
        err = np.abs(gi - fw.image[v]).max(0)
        assert err[ok].max() <= IMG_TOL if ok.any() else True
        assert np.abs(gT - fw.T[v])[ok].max() <= IMG_TOL
        exp_n = gpu_n_contrib(fw, v, kept)
        bad_n = int((gn != exp_n)[ok].sum())
        assert bad_n == 0, f"view {v}: n_contrib differs on {bad_n} pixels not explained by a flip"
    say(f"[gpu] {name}: pixels beyond 1e-4: {total_bad}, unexplained: {total_unexp}")
    assert total_unexp == 0
    r.close()


@pytest.mark.parametrize("name", list(SCENES))
def test_backward_parity(name):
    sc, fw = case(name)
    say(f"[gpu] render_bwd {name}")
    rng = np.random.default_rng(123)
    targets = {v: rng.uniform(0, 1, fw.image[v].shape) for v in fw.views}
    L, G = fw.loss(targets)
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    imgs = gpu_images(r)
    flips = {}
    for v in range(len(sc.cams)):
        fl, unexp, _ = explain(fw, v, imgs[v][0], imgs[v][1])
        assert not unexp
        if fl:
            flips[v] = fl
    g_flat = np.concatenate([G[v].reshape(-1) for v in fw.views]).astype(np.float32)
    gt = torch.from_numpy(g_flat).to("cuda:0")
    r.backward(gt)
    torch.cuda.synchronize()
    ref_atlas, ref_g2 = fw.backward(G, flips=flips)
    got = r.dL_datlas.cpu().numpy().reshape(sc.frames, sc.C, sc.H, sc.W)
    occ = sc.occupancy.astype(bool)
    assert np.all(got[:, :, ~occ] == 0.0)
    # per (view, Gaussian) 2D gradients
    g2 = r.sets[0].grad2d[:9 * r.sets[0].info.n_gv].cpu().numpy().reshape(9, len(sc.cams), r.N)
    for v in range(len(sc.cams)):
        st = grad_compare(g2[:, v, :][None], ref_g2[v].T[None])
        say(f"[gpu] {name} view {v} grad2d: {st}")
        assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st
    st = grad_compare(got.reshape(sc.frames, sc.C, -1)[:, :, occ.reshape(-1)],
                      ref_atlas.reshape(sc.frames, sc.C, -1)[:, :, occ.reshape(-1)])
    say(f"[gpu] {name} dL/datlas: {st}")
    assert st["n_bad"] == 0 and st["worst_l2"] <= 1e-3, st
    r.close()


def test_loss_l1_parity():
    sc, fw = case("tiny")
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    rng = np.random.default_rng(5)
    tgt = rng.uniform(0, 1, 3 * r.n_pixels).astype(np.float32)
    loss = float(r.loss_l1(torch.from_numpy(tgt).to("cuda:0")).item())
    img = r.image.cpu().numpy().astype(np.float64)
    L, G = oracle.loss_l1(img, tgt.astype(np.float64))
    assert abs(loss - L) <= 1e-6 * max(1.0, L)
    np.testing.assert_array_equal(r.dL_dimage.cpu().numpy(), G.astype(np.float32))
    r.close()


@pytest.mark.parametrize("name", ["multiframe", "odd_atlas"])
def test_adam_parity(name):
    """Sparse Adam against the oracle over three steps: a 10 x 10 atlas
    (16-byte texel quads) and a 9 x 9 one (one texel per thread)."""
    if name == "odd_atlas":
        sc = synth.random_scene(side=9, sh_degree=1, views=2, width=64, height=50, seed=9, frames=2,
                                occupancy=0.8, lscale=(-2.7, 0.5))
        fw = oracle.Forward(sc)
    else:
        sc, fw = case(name)
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    rng = np.random.default_rng(6)
    g = rng.standard_normal(atlas.numel()).astype(np.float32)
    r.dL_datlas.copy_(torch.from_numpy(g))
    p = sc.atlas.reshape(-1).astype(np.float64).copy()
    m = np.zeros_like(p)
    vv = np.zeros_like(p)
    vis_g = fw.visible()                                     # (F, N)
    vis_t = np.zeros((sc.frames, sc.H * sc.W), np.uint8)
    vis_t[:, fw.ids] = vis_g
    vis_e = np.broadcast_to(vis_t[:, None, :], (sc.frames, sc.C, sc.H * sc.W)).reshape(-1)
    for step in (1, 2, 3):
        r.adam_step(atlas, lr=1e-2)
        oracle.adam(p, g.astype(np.float64), m, vv, np.ascontiguousarray(vis_e), 1e-2, 0.9, 0.999, 1e-8, step)
    got = atlas.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, p, rtol=1e-5, atol=1e-6)
    r.close()


def test_tile_shape_and_batch_invariance():
    sc, fw = case("ragged")
    ref = None
    for tiling in [(16, 16, 256), (16, 16, 64), (8, 32, 128), (32, 8, 256), (32, 8, 64)]:
        say(f"[gpu] tiling {tiling}")
        r = renderer(sc, tiling=tiling)
        run_forward(r, atlas_tensor(sc))
        img = r.image.cpu().numpy()
        if ref is None:
            ref = img
        else:
            assert np.array_equal(img, ref), f"image differs for tiling {tiling}"
        r.close()


def test_batched_equals_plain():
    sc, fw = case("tiny")
    atlas = atlas_tensor(sc)
    out = []
    for batched in (True, False):
        say(f"[gpu] batched={batched}")
        r = renderer(sc, batched=batched)
        run_forward(r, atlas)
        rng = np.random.default_rng(7)
        tgt = torch.from_numpy(rng.uniform(0, 1, 3 * r.n_pixels).astype(np.float32)).to("cuda:0")
        r.loss_l1(tgt)
        r.backward()
        torch.cuda.synchronize()
        out.append((r.image.cpu().numpy(), r.dL_datlas.cpu().numpy()))
        r.close()
    assert np.array_equal(out[0][0], out[1][0])
    st = grad_compare(out[1][1].reshape(sc.frames, sc.C, -1), out[0][1].reshape(sc.frames, sc.C, -1), rel=1e-4)
    assert st["n_bad"] == 0, st


def test_empty_atlas_renders_background():
    sc = synth.random_scene(side=4, sh_degree=0, views=2, width=40, height=24, seed=0)
    sc.occupancy[:] = 0
    sc.atlas[:] = 0
    sc.bg = (0.1, 0.2, 0.3)
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    img = r.image.cpu().numpy().reshape(-1)
    for v, c in enumerate(sc.cams):
        im = img[3 * r.pix_base[v]:3 * r.pix_base[v + 1]].reshape(3, c.height, c.width)
        for ch in range(3):
            assert np.all(im[ch] == np.float32(sc.bg[ch]))
    r.backward(torch.ones(3 * r.n_pixels, device="cuda:0"))
    assert float(r.dL_datlas.abs().max().item()) == 0.0
    r.close()


def test_capacity_overflow_is_reported_and_recovered():
    """The raw protocol (forward with check=False): pg_status_check reports the
    overflow and the count that suffices, growing to it renders the step."""
    sc, fw = case("tiny")
    r = renderer(sc, cap=16)
    r.forward(atlas_tensor(sc), check=False)
    s = r.sets[0]
    [(ovf, need)] = r.status()
    assert ovf and int(s.overflow.item()) == 1
    assert need == int(r.bin_records()["n_tiles"].astype(np.int64).sum())   # the count that suffices
    assert r.grow_capacity(1.0) and s.cap == need
    r.forward(atlas_tensor(sc), check=False)
    assert r.status() == [(False, need)]
    img = gpu_images(r)
    for v in fw.views:
        flips, unexp, _ = explain(fw, v, img[v][0], img[v][1])
        assert not unexp
        ok = np.ones(img[v][2].shape, bool)
        ok.reshape(-1)[list(flips)] = False
        assert np.abs(img[v][0] - fw.image[v]).max(0)[ok].max() <= IMG_TOL
    r.close()


def test_gradients_bitwise_deterministic():
    """No floating-point atomics: two adjoint runs give identical bits."""
    sc, fw = case("ragged")
    r = renderer(sc)
    atlas = atlas_tensor(sc)
    run_forward(r, atlas)
    g = torch.from_numpy(np.random.default_rng(3).standard_normal(3 * r.n_pixels).astype(np.float32)).to("cuda:0")
    outs = []
    for _ in range(3):
        r.backward(g)
        torch.cuda.synchronize()
        outs.append((r.dL_datlas.clone(), r.sets[0].grad2d.clone()))
    for a, b in outs[1:]:
        assert torch.equal(a, outs[0][0]) and torch.equal(b, outs[0][1])
    r.close()


def test_eager_forward_grows_after_an_overflow():
    """An eager forward that overflows grows the buffers to the reported
    count (with headroom) and renders again: the image is never the
    background an overflowed sort leaves."""
    sc, fw = case("ragged")
    r = renderer(sc, cap=16)
    r.forward(atlas_tensor(sc))
    torch.cuda.synchronize()
    [(ovf, need)] = r.status()
    assert not ovf and r.sets[0].cap >= need > 16
    img = gpu_images(r)
    for v in fw.views:
        flips, unexp, _ = explain(fw, v, img[v][0], img[v][1])
        assert not unexp
    r.close()


def test_workspace_plan_matches_the_buffers():
    """pg_workspace_query (host only) gives the sizes of the buffers the
    step's calls take: they agree with what the per-stage queries and the
    renderer's allocations use."""
    sc, fw = case("ragged")
    r = renderer(sc)
    run_forward(r, atlas_tensor(sc))
    s = r.sets[0]
    plan = r.plan()
    n_gv, T, P = s.info.n_gv, s.info.n_tiles, r.n_pixels
    nb = lambda t: t.numel() * t.element_size()   # noqa: E731
    assert plan["fetch_ws"] == r.fetch_ws_bytes and plan["sort_ws"] == s.ws_bytes
    assert plan["splats"] == 48 * n_gv == nb(s.splats) and plan["bins"] == 16 * n_gv == nb(s.bins)
    assert plan["tile_sets"] == nb(s.tiles) and plan["inst_first"] == nb(s.inst_first)
    assert plan["keys"] == nb(s.keys) and plan["values"] == nb(s.values) and plan["entries"] == nb(s.entries)
    assert plan["inst_grad"] == nb(s.inst_grad) and plan["grad2d"] == nb(s.grad2d)
    assert plan["tile_ranges"] == 8 * T == nb(s.ranges) and plan["tile_order"] == nb(s.order)
    assert plan["image"] == 12 * P == nb(r.image) and plan["final_T"] == nb(r.final_T)
    assert plan["n_contrib"] == nb(r.n_contrib) and plan["dL_dimage"] == nb(r.dL_dimage)
    assert plan["dL_datlas"] == nb(r.dL_datlas) and plan["params"] == nb(r.params)
    assert plan["texel_gauss"] == nb(r.texel_gauss) and plan["visible"] == nb(r.visible)
    parts = [v for k, v in plan.items() if k != "total"]
    assert plan["total"] == sum((v + 255) // 256 * 256 for v in parts)
    big = r.plan(inst_capacity=10 * s.cap)
    assert big["keys"] == 10 * plan["keys"] and big["sort_ws"] >= plan["sort_ws"]
    r.close()
