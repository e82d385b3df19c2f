"""Pins of the oracle's covariance-aware flow masking (Sec. 4.2 masking
paragraph, Algorithm 1): a Gaussian is dynamic for a camera when a pixel of
its 3-sigma ellipse carries motion; the labels of several cameras are OR-ed.

Checked against: the closed form of an isotropic Gaussian on the optical
axis (its ellipse is a disc of radius 3 sqrt(f^2 sigma^2 / z^2 + 0.3)), a
brute force over every pixel of the image with numpy, the OR across cameras,
and empty / full masks."""
import math

import numpy as np

import oracle
import synth

F_128 = synth.focal_for_hfov(128)


def one_gaussian(mu, lscale, L=0):
    P = np.zeros((synth.n_channels(L), 1), np.float64)
    P[0:3, 0] = mu
    P[3:6, 0] = lscale
    P[6, 0] = 1.0
    return P


def test_disc_closed_form():
    """Isotropic on-axis Gaussian: mean (64, 64), q = d^2 / v with
    v = f^2 sigma^2 / z^2 + 0.3.  A one-pixel mask marks it dynamic exactly
    when that pixel's centre is within 3 sqrt(v) of the mean."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 128, 128)
    z, sigma = 3.0, 0.02
    v = F_128 ** 2 * sigma ** 2 / z ** 2 + 0.3
    R = 3 * math.sqrt(v)
    P = one_gaussian((0.0, 0.0, z), [math.log(sigma)] * 3)
    checked = {True: 0, False: 0}
    for px in range(64, 64 + int(R) + 3):
        for py in (64, 66, 70):
            d2 = (px + 0.5 - 64) ** 2 + (py + 0.5 - 64) ** 2
            if abs(d2 / v - 9) < 1e-6:
                continue                       # too close to the boundary to call
            m = np.zeros((128, 128), np.uint8)
            m[py, px] = 1
            D = oracle.flow_mask(P, 0, cam, m)
            inside = d2 / v <= 9
            assert D[0] == int(inside), (px, py, d2 / v)
            checked[inside] += 1
    assert checked[True] >= 3 and checked[False] >= 3


def brute(P, L, cam, mask):
    pr = oracle.project(P, L, cam, 16, 16)
    H, W = mask.shape
    ys, xs = np.nonzero(mask)
    cx, cy = xs + 0.5, ys + 0.5
    out = np.zeros(P.shape[1], np.uint8)
    for i, g in enumerate(pr):
        if g["radius"] <= 0 or not len(xs):
            continue
        a, b, c = g["conic"]
        dx, dy = cx - g["mean"][0], cy - g["mean"][1]
        q = (a * dx * dx + 2.0 * b * dx * dy) + c * dy * dy
        out[i] = np.any(q <= 9.0)
    return out


def random_mask(rng, H, W, n_discs=6):
    m = np.zeros((H, W), np.uint8)
    yy, xx = np.mgrid[0:H, 0:W]
    for _ in range(n_discs):
        cx, cy, r = rng.uniform(0, W), rng.uniform(0, H), rng.uniform(2, 12)
        m[(xx - cx) ** 2 + (yy - cy) ** 2 <= r * r] = 1
    return m


def test_matches_brute_force_over_every_pixel_and_ors_cameras():
    sc = synth.random_scene(side=14, sh_degree=1, views=3, width=90, height=70, seed=21, lscale=(-2.6, 0.6))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    rng = np.random.default_rng(8)
    total = np.zeros(params.shape[2], np.uint8)
    expect_total = np.zeros_like(total)
    some = False
    for cam in sc.cams:
        m = random_mask(rng, cam.height, cam.width)
        D = oracle.flow_mask(params[0], sc.sh_degree, cam, m)
        E = brute(params[0], sc.sh_degree, cam, m)
        assert np.array_equal(D, E)
        some |= bool(D.any()) and not bool(D.all())
        oracle.flow_mask(params[0], sc.sh_degree, cam, m, total)
        expect_total |= E
    assert some, "the masks must split the Gaussians"
    assert np.array_equal(total, expect_total)


def test_empty_and_full_masks():
    sc = synth.random_scene(side=10, sh_degree=0, views=1, width=64, height=48, seed=22, lscale=(-2.8, 0.5))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    cam = sc.cams[0]
    zero = np.zeros((cam.height, cam.width), np.uint8)
    assert not oracle.flow_mask(params[0], 0, cam, zero).any()
    full = np.ones_like(zero)
    D = oracle.flow_mask(params[0], 0, cam, full)
    assert np.array_equal(D, brute(params[0], 0, cam, full))
    # full mask: dynamic exactly when a pixel centre of the image lies in the ellipse,
    # which implies the Gaussian is drawn (listed in a kept tile)
    pr = oracle.project(params[0], 0, cam, 16, 16)
    assert np.all(pr["valid"][D == 1] == 1)
