"""Pins for the oracle's compositing, adjoint, loss and Adam.

Closed forms of the compositing formula C = sum_i T_i alpha_i c_i with
T_i = prod_{j<i}(1 - alpha_j) (supplementary, viewer section), brute force
(no tiles) against the tiled walk, tile-shape invariance, frozen-decision
finite differences for the adjoint, and textbook L1 / Adam.
"""
import math

import numpy as np
import pytest

import oracle
import synth

C0 = 0.5 / math.sqrt(math.pi)


def scene_from_gaussians(gs, cam, sh_degree=0, tiling=(16, 16)):
    """gs: list of dicts(mu, ls, q, lo, rgb) -> Scene with a 1 x n atlas."""
    n = len(gs)
    C = synth.n_channels(sh_degree)
    atlas = np.zeros((1, C, 1, n), np.float32)
    for i, g in enumerate(gs):
        atlas[0, 0:3, 0, i] = g["mu"]
        atlas[0, 3:6, 0, i] = g.get("ls", (-3.0, -3.0, -3.0))
        atlas[0, 6:10, 0, i] = g.get("q", (1.0, 0.0, 0.0, 0.0))
        atlas[0, 10, 0, i] = g.get("lo", 0.0)
        rgb = np.asarray(g.get("rgb", (0.5, 0.5, 0.5)))
        atlas[0, 11:14, 0, i] = (rgb - 0.5) / C0
    return synth.Scene("manual", atlas, np.ones((1, n), np.uint8), [cam], sh_degree,
                       synth.Tiling(tiling[0], tiling[1], 64))


def logit(o):
    return math.log(o / (1 - o))


def tile_list_lengths(fw, v):
    """Length of the tile list of every pixel of view v."""
    cam = fw.scene.cams[v]
    TX = (cam.width + fw.tw - 1) // fw.tw
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    t = (ys // fw.th) * TX + xs // fw.tw
    return (fw.ranges[v][t, 1] - fw.ranges[v][t, 0]).astype(np.int32)


def test_single_gaussian_closed_form():
    cam = synth.pinhole(np.eye(3), np.zeros(3), 64, 48)
    z, sigma, o = 3.0, 0.03, 0.8
    rgb = np.array([0.9, 0.2, 0.6], np.float32)
    sc = scene_from_gaussians([dict(mu=(0, 0, z), ls=[math.log(sigma)] * 3, lo=logit(o), rgb=rgb)], cam)
    fw = oracle.Forward(sc)
    o = 1 / (1 + math.exp(-np.float32(logit(o))))
    sig = np.float64(np.float32(math.log(sigma)))
    v = cam.fx ** 2 * math.exp(2 * sig) / z ** 2 + 0.3
    ys, xs = np.mgrid[0:48, 0:64]
    q = ((xs + 0.5 - 32) ** 2 + (ys + 0.5 - 24) ** 2) / v
    alpha = np.minimum(0.99, o * np.exp(-q / 2))
    on = (q <= 9) & (alpha >= 1 / 255)
    col = 0.5 + C0 * sc.atlas[0, 11:14, 0, 0].astype(np.float64)
    expect = np.where(on[None], alpha[None] * col[:, None, None], 0.0)
    np.testing.assert_allclose(fw.image[0], expect, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(fw.T[0], np.where(on, 1 - alpha, 1.0), rtol=1e-12)
    # T never drops below 1e-4 (alpha <= 0.99), so every pixel reaches the end of its
    # tile's list: one Gaussian where the tile lists it, which includes every lit pixel
    tl = tile_list_lengths(fw, 0)
    assert np.array_equal(fw.n[0], tl) and np.all(tl[on] == 1)


@pytest.mark.parametrize("o,k", [(0.5, 5), (0.5, 20), (0.9, 8), (0.3, 40)])
def test_stacked_transmittance_product(o, k):
    """k identical Gaussians centred on a pixel centre: C = c (1 - (1-o)^n),
    n = min(k, n*), n* = largest n with (1 - o)^n >= 1e-4; n is also the
    pixel's n_contrib (it stops before Gaussian n* when k > n*, else reaches
    the end of its list of k)."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 16, 16)
    cam.cx = cam.cy = 8.5  # principal point on the centre of pixel (8, 8)
    lo = np.float32(logit(o))
    of = 1 / (1 + math.exp(-float(lo)))
    gs = [dict(mu=(0, 0, 3.0), ls=(-4, -4, -4), lo=lo, rgb=(0.7, 0.3, 0.1)) for _ in range(k)]
    sc = scene_from_gaussians(gs, cam)
    fw = oracle.Forward(sc)
    nstar = 0
    while (1 - of) ** (nstar + 1) >= 1e-4:
        nstar += 1
    n = min(k, nstar)
    col = 0.5 + C0 * sc.atlas[0, 11:14, 0, 0].astype(np.float64)
    np.testing.assert_allclose(fw.image[0][:, 8, 8], col * (1 - (1 - of) ** n), rtol=1e-12)
    assert math.isclose(fw.T[0][8, 8], (1 - of) ** n, rel_tol=1e-12)
    assert fw.n[0][8, 8] == n


def test_two_gaussians_closed_form_and_adjoint():
    """1x1 image; two Gaussians on the axis through the pixel centre at depths 2 and 3.
    C = a1 c1 + (1 - a1) a2 c2 (bg 0); dC/da1 = c1 - a2 c2, dC/da2 = (1 - a1) c2, dC/dc1 = a1."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 1, 1)
    cam.cx = cam.cy = 0.5
    o1, o2 = 0.6, 0.7
    c1, c2 = np.array([0.9, 0.1, 0.4]), np.array([0.2, 0.8, 0.5])
    gs = [dict(mu=(0, 0, 3.0), lo=logit(o2), rgb=c2), dict(mu=(0, 0, 2.0), lo=logit(o1), rgb=c1)]
    fw = oracle.Forward(scene_from_gaussians(gs, cam))
    pr = fw.proj[0]
    a2, a1 = pr["opacity"]
    c2f, c1f = pr["color"]
    np.testing.assert_allclose(fw.image[0][:, 0, 0], a1 * c1f + (1 - a1) * a2 * c2f, rtol=1e-14)
    for ch in range(3):
        G = np.zeros((3, 1, 1))
        G[ch] = 1.0
        g2 = oracle.backward_view(pr, cam, 16, 16, fw.inst[0], fw.ranges[0], G)
        # q = 0 at the pixel centre, so dL/do = dL/dalpha
        np.testing.assert_allclose(g2[1, 5], c1f[ch] - a2 * c2f[ch], rtol=1e-13)
        np.testing.assert_allclose(g2[0, 5], (1 - a1) * c2f[ch], rtol=1e-13)
        np.testing.assert_allclose(g2[1, 6 + ch], a1, rtol=1e-13)
        np.testing.assert_allclose(g2[0, 6 + ch], (1 - a1) * a2, rtol=1e-13)


def test_alpha_clamp_has_zero_opacity_gradient():
    cam = synth.pinhole(np.eye(3), np.zeros(3), 1, 1)
    cam.cx = cam.cy = 0.5
    fw = oracle.Forward(scene_from_gaussians([dict(mu=(0, 0, 2.0), lo=6.0)], cam))
    assert fw.image[0][0, 0, 0] == pytest.approx(0.99 * fw.proj[0]["color"][0][0])
    g2 = oracle.backward_view(fw.proj[0], cam, 16, 16, fw.inst[0], fw.ranges[0], np.ones((3, 1, 1)))
    assert g2[0, 5] == 0.0 and g2[0, 2] == 0.0 and g2[0, 0] == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiled_equals_brute_force_bitwise(seed):
    sc = synth.random_scene(side=12, sh_degree=1, views=3, width=72, height=56, seed=seed, lscale=(-2.8, 0.5))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    for cam in sc.cams:
        pr = oracle.project(params[0], 1, cam, 16, 16)
        inst, ranges = oracle.bin_sort(pr, cam, 16, 16)
        img, T, n, _ = oracle.render(pr, cam, 16, 16, inst, ranges)
        bimg, bT, bn = oracle.render_brute(pr, cam)
        assert np.array_equal(img, bimg) and np.array_equal(T, bT)
        # a pixel stops before the end of its tile list exactly when it stops
        # before the end of the full list (the Gaussians it composites are the same)
        TX = (cam.width + 15) // 16
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        t = (ys // 16) * TX + xs // 16
        tl = ranges[t, 1] - ranges[t, 0]
        m = int((pr["radius"] > 0).sum())
        assert np.all(n <= tl) and np.all(bn <= m)
        assert np.array_equal(n < tl, bn < m)
        assert img.max() > 0.05


def test_image_independent_of_tile_shape():
    sc = synth.random_scene(side=14, sh_degree=0, views=2, width=80, height=64, seed=9, lscale=(-2.6, 0.5))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    for cam in sc.cams:
        ref = None
        for tw, th in ((16, 16), (8, 32), (32, 8)):
            pr = oracle.project(params[0], 0, cam, tw, th)
            inst, ranges = oracle.bin_sort(pr, cam, tw, th)
            img, T, _, _ = oracle.render(pr, cam, tw, th, inst, ranges)
            if ref is None:
                ref = (img, T)
            else:
                assert np.array_equal(img, ref[0]) and np.array_equal(T, ref[1])


def test_background_enters_through_final_transmittance():
    sc = synth.random_scene(side=8, sh_degree=0, views=1, width=48, height=40, seed=3, lscale=(-2.5, 0.4))
    bg = (0.25, 0.5, 1.0)
    a = oracle.Forward(sc)
    b = oracle.Forward(sc, bg=bg)
    np.testing.assert_allclose(b.image[0] - a.image[0], np.asarray(bg)[:, None, None] * a.T[0][None], atol=1e-15)


def test_empty_scene_renders_background():
    sc = synth.random_scene(side=4, sh_degree=0, views=1, width=32, height=32, seed=0)
    sc.occupancy[:] = 0
    sc.atlas[:] = 0
    fw = oracle.Forward(sc, bg=(0.1, 0.2, 0.3))
    np.testing.assert_array_equal(fw.image[0], np.broadcast_to(np.array([0.1, 0.2, 0.3])[:, None, None], (3, 32, 32)))
    assert np.all(fw.n[0] == 0)


# ------------------------------------------------------------------ adjoint vs finite differences

def _fd_scene(seed, sh_degree, views=2, frames=1):
    return synth.random_scene(side=6, sh_degree=sh_degree, views=views, width=48, height=40, seed=seed,
                              lscale=(-2.6, 0.4), frames=frames)


@pytest.mark.parametrize("seed,L", [(11, 0), (12, 1), (13, 3)])
def test_adjoint_matches_frozen_finite_differences(seed, L):
    sc = _fd_scene(seed, L)
    fw = oracle.Forward(sc)
    rng = np.random.default_rng(seed)
    G = {v: rng.standard_normal(fw.image[v].shape) for v in fw.views}
    gA, _ = fw.backward(G)
    C = sc.C
    gflat = gA[0].reshape(C, -1)[:, fw.ids]
    vis = fw.visible()[0]
    checked = 0
    for i in np.flatnonzero(vis)[:6]:
        for ch in range(C):
            h = 1e-6
            fd = fw.fd(G, 0, i, ch, h)
            an = gflat[ch, i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, ch, fd, an)
            checked += 1
    assert checked > 0
    # invisible Gaussians get exactly zero
    for i in np.flatnonzero(vis == 0):
        assert np.all(gflat[:, i] == 0.0)


def test_frozen_fd_equals_plain_fd_away_from_decision_boundaries():
    """The frozen-decision difference is checked against re-rendering the whole
    scene from a perturbed atlas (plain central difference)."""
    sc = _fd_scene(21, 1, views=1)
    fw = oracle.Forward(sc)
    rng = np.random.default_rng(0)
    G = {0: rng.standard_normal(fw.image[0].shape)}
    i = int(np.flatnonzero(fw.visible()[0])[0])
    texel = fw.ids[i]
    h = 1e-4
    for ch in (0, 1, 4, 7, 10, 12):
        fz = fw.fd(G, 0, i, ch, h)
        vals = []
        for s in (+1, -1):
            sc2 = synth.Scene(sc.name, sc.atlas.copy(), sc.occupancy, sc.cams, sc.sh_degree, sc.tiling)
            # perturb in float64 through the oracle's parameter planes: rebuild from params
            f2 = oracle.Forward(sc2)
            P = f2.params[0].copy()
            P[ch, i] += s * h
            pr = oracle.project(P, sc.sh_degree, sc.cams[0], f2.tw, f2.th)
            inst, ranges = oracle.bin_sort(pr, sc.cams[0], f2.tw, f2.th)
            img, _, _, _ = oracle.render(pr, sc.cams[0], f2.tw, f2.th, inst, ranges)
            vals.append(float((G[0] * img).sum()))
        plain = (vals[0] - vals[1]) / (2 * h)
        assert abs(plain - fz) <= 1e-6 * max(1.0, abs(fz)), (ch, plain, fz)
    assert texel == fw.ids[i]


def test_dynamic_mask_freezes_static_gaussians():
    sc = synth.random_scene(side=6, sh_degree=0, views=2, width=48, height=40, seed=31, lscale=(-2.6, 0.4),
                            dynamic_frac=0.5)
    fw = oracle.Forward(sc)
    G = {v: np.ones_like(fw.image[v]) for v in fw.views}
    gA, _ = fw.backward(G)
    gfree, _ = fw.backward(G, dynamic=None)
    dyn = sc.dynamic.astype(bool)
    assert np.all(gA[0][:, ~dyn] == 0)
    np.testing.assert_array_equal(gA[0][:, dyn], gfree[0][:, dyn])


# ------------------------------------------------------------------ loss / Adam

def test_l1_loss_textbook():
    a = np.array([0.5, 0.2, 0.7, 0.1])
    b = np.array([0.4, 0.2, 0.9, 0.0])
    L, G = oracle.loss_l1(a, b)
    assert L == pytest.approx((0.1 + 0 + 0.2 + 0.1) / 4)
    np.testing.assert_array_equal(G, np.array([1, 0, -1, 1]) / 4)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    vis = (rng.random(50) < 0.7).astype(np.uint8)
    p1, m, v = p.copy(), np.zeros(50), np.zeros(50)
    oracle.adam(p1, g, m, v, vis, 1e-3, 0.9, 0.999, 1e-8, 1)
    exp = np.where(vis > 0, p - 1e-3 * g / (np.abs(g) + 1e-8), p)
    np.testing.assert_allclose(p1, exp, rtol=1e-12)
    # second step against the textbook recursion
    g2 = rng.standard_normal(50)
    oracle.adam(p1, g2, m, v, vis, 1e-3, 0.9, 0.999, 1e-8, 2)
    m_ = 0.9 * (0.1 * g) + 0.1 * g2
    v_ = 0.999 * (0.001 * g * g) + 0.001 * g2 * g2
    step = 1e-3 * (m_ / (1 - 0.81)) / (np.sqrt(v_ / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(p1, np.where(vis > 0, exp - step, p), rtol=1e-10)
