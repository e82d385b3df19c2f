"""Pins of the oracle's full objective (Sec. 4.2 "Objective"): SSIM and its
gradient, the photometric blend with L1, and the scale / opacity
regularisers.

Checked against: SSIM(x, x) = 1 with zero gradient; constant planes against
the closed form (2ab + C1) / (a^2 + b^2 + C1) away from the border; the
window statistics recomputed with scipy.ndimage.correlate (zero padding);
symmetry in its arguments; central differences of the oracle's own sums for
every gradient; hand-evaluated regulariser values; the blend's two ends
(L1 alone, 1 - SSIM alone)."""
import math

import numpy as np
from scipy import ndimage

import oracle

C1, C2 = 0.01 ** 2, 0.03 ** 2


def window():
    k = np.arange(11) - 5.0
    g = np.exp(-(k * k) / (2 * 1.5 ** 2))
    g /= g.sum()
    return np.outer(g, g)


def test_ssim_of_a_plane_with_itself_is_one_with_zero_gradient():
    x = np.random.default_rng(0).uniform(0, 1, (23, 31))
    tot, g, m = oracle.ssim(x, x, grad=True, smap=True)
    assert np.allclose(m, 1.0, rtol=0, atol=1e-12) and abs(tot - x.size) < 1e-9
    assert np.abs(g).max() < 1e-9


def test_constant_planes_closed_form_in_the_interior():
    for a, b in ((0.3, 0.7), (0.9, 0.1), (0.5, 0.5)):
        x = np.full((25, 27), a)
        y = np.full((25, 27), b)
        _, m = oracle.ssim(x, y, smap=True)
        inner = m[5:-5, 5:-5]
        assert np.allclose(inner, (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12)


def test_window_statistics_against_scipy():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0, 1, (2, 19, 26))
    w = window()
    mu_x = ndimage.correlate(x, w, mode="constant")
    mu_y = ndimage.correlate(y, w, mode="constant")
    exx = ndimage.correlate(x * x, w, mode="constant")
    eyy = ndimage.correlate(y * y, w, mode="constant")
    exy = ndimage.correlate(x * y, w, mode="constant")
    ref = ((2 * mu_x * mu_y + C1) * (2 * (exy - mu_x * mu_y) + C2)) / (
        (mu_x ** 2 + mu_y ** 2 + C1) * ((exx - mu_x ** 2) + (eyy - mu_y ** 2) + C2))
    _, m = oracle.ssim(x, y, smap=True)
    np.testing.assert_allclose(m, ref, rtol=1e-11, atol=1e-13)
    _, m2 = oracle.ssim(y, x, smap=True)
    np.testing.assert_allclose(m2, m, rtol=1e-12, atol=1e-14)


def test_ssim_gradient_central_differences():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(0, 1, (2, 17, 21))
    _, g = oracle.ssim(x, y, grad=True)
    h = 1e-6
    for (i, j) in [(0, 0), (8, 10), (16, 20), (3, 15), (12, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[i, j] += h
        xm[i, j] -= h
        fd = (oracle.ssim(xp, y) - oracle.ssim(xm, y)) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[i, j])


def test_photometric_blend_ends_and_gradient():
    rng = np.random.default_rng(3)
    imgs = {0: rng.uniform(0, 1, (3, 14, 18)), 1: rng.uniform(0, 1, (3, 9, 12))}
    tgts = {v: rng.uniform(0, 1, im.shape) for v, im in imgs.items()}
    n = sum(im.size for im in imgs.values())
    L0, G0 = oracle.photo_loss(imgs, tgts, 0.0)
    l1 = sum(np.abs(imgs[v] - tgts[v]).sum() for v in imgs) / n
    assert abs(L0 - l1) < 1e-14
    for v in imgs:
        assert np.array_equal(G0[v], np.sign(imgs[v] - tgts[v]) / n)
    L1, _ = oracle.photo_loss(imgs, tgts, 1.0)
    s = sum(oracle.ssim(imgs[v][c], tgts[v][c]) for v in imgs for c in range(3))
    assert abs(L1 - (1 - s / n)) < 1e-14
    lam = 0.2
    L, G = oracle.photo_loss(imgs, tgts, lam)
    h = 1e-7
    for (v, c, i, j) in [(0, 0, 3, 4), (1, 2, 8, 11), (0, 1, 0, 17)]:
        ip = {k: a.copy() for k, a in imgs.items()}
        im = {k: a.copy() for k, a in imgs.items()}
        ip[v][c, i, j] += h
        im[v][c, i, j] -= h
        fd = (oracle.photo_loss(ip, tgts, lam)[0] - oracle.photo_loss(im, tgts, lam)[0]) / (2 * h)
        assert abs(fd - G[v][c, i, j]) <= 1e-6 * abs(fd), (v, c, i, j)


def test_regularisers_hand_values_and_gradients():
    F, C, N = 2, 14, 3
    P = np.zeros((F, C, N))
    P[0, 3:6, 0] = np.log([0.5, 2.0, 1.0])      # max scale 2.0 > s_max 1.5: hinge 0.5 on channel 4
    P[0, 3:6, 1] = np.log([0.1, 0.2, 0.3])      # under s_max
    P[1, 3:6, 2] = np.log([3.0, 1.0, 1.0])      # hinge 1.5 on channel 3
    P[:, 10, :] = [[0.0, 2.0, -1.0], [0.5, -3.0, 1.0]]
    s_max = 1.5
    Ls, Lo, g, n = oracle.regularisers(P, s_max)
    assert n == 6
    assert math.isclose(Ls, (0.5 ** 2 + 1.5 ** 2) / 6, rel_tol=1e-14)
    o = 1 / (1 + np.exp(-P[:, 10, :]))
    assert math.isclose(Lo, float((o * (1 - o)).sum()) / 6, rel_tol=1e-14)
    # only the dynamic ones
    dyn = np.array([[1, 0, 0], [0, 0, 1]], np.uint8)
    Ls2, Lo2, g2, n2 = oracle.regularisers(P, s_max, dyn=dyn)
    assert n2 == 2 and math.isclose(Ls2, (0.25 + 2.25) / 2, rel_tol=1e-14)
    assert np.all(g2[0, :, 1] == 0) and np.all(g2[1, :, 0] == 0)
    # central differences of w_s L_scale + w_o L_opacity
    ws, wo = 0.7, 1.3
    _, _, g, _ = oracle.regularisers(P, s_max, ws, wo)
    h = 1e-6
    for idx in [(0, 4, 0), (1, 3, 2), (0, 10, 1), (1, 10, 0), (0, 3, 1)]:
        Pp, Pm = P.copy(), P.copy()
        Pp[idx] += h
        Pm[idx] -= h
        fp = oracle.regularisers(Pp, s_max)
        fm = oracle.regularisers(Pm, s_max)
        fd = (ws * (fp[0] - fm[0]) + wo * (fp[1] - fm[1])) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 + 1e-6 * abs(fd), (idx, fd, g[idx])
