"""Pins for the oracle's near-threshold machinery: the decisions whose FP64
margin lies inside a guard band are reported ("near"), and a flip takes such
a decision the other way, in the forward walk and in the adjoint.

The three compositing decisions (the d^2 <= 9 footprint of Sec. 4.2 and
Alg. 1 step 5; the alpha skip and the termination of the 3DGS rasteriser the
paper names in Sec. 3) are each put just inside and just outside the band on
hand-built scenes:

  * q:  an isotropic Gaussian on the optical axis, whose on-axis closed form
        Sigma2D = (f^2 s^2 / z^2 + 0.3) I gives q at a chosen pixel centre;
  * alpha: a Gaussian centred on a pixel centre (q = 0, alpha = o) with the
        opacity at 1/255 (1 + eps);
  * T': three Gaussians stacked on a pixel centre, the third taking T below
        or above 1e-4 by a relative eps.

Expected values are evaluated by hand from the FP32 texel values (not read
from the oracle's projection).  The adjoint under flips is checked against
hand-evaluated derivatives, against central differences of the flipped
forward walk, and against the unflipped adjoint of the same scene moved to
the other side of the threshold.
"""
import math

import numpy as np
import pytest

import oracle
import synth

C0 = 0.5 / math.sqrt(math.pi)
BAND = 1e-4
INSIDE, OUTSIDE = 3e-5, 3e-4          # relative offsets from a threshold


def logit(o):
    return math.log(o / (1.0 - o))


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def scene(gs, cam):
    """gs: dicts(mu, ls, lo, rgb) -> one-frame scene with a 1 x n atlas (SH degree 0)."""
    n = len(gs)
    atlas = np.zeros((1, synth.n_channels(0), 1, n), np.float32)
    for i, g in enumerate(gs):
        atlas[0, 0:3, 0, i] = g["mu"]
        atlas[0, 3:6, 0, i] = g.get("ls", (-3.0,) * 3)
        atlas[0, 6:10, 0, i] = (1.0, 0.0, 0.0, 0.0)
        atlas[0, 10, 0, i] = g["lo"]
        atlas[0, 11:14, 0, i] = (np.asarray(g.get("rgb", (0.6, 0.4, 0.2))) - 0.5) / C0
    return synth.Scene("flips", atlas, np.ones((1, n), np.uint8), [cam], 0, synth.Tiling(16, 16, 64))


def colour(sc, i):
    """Degree-0 colour max(0, 0.5 + k0 / (2 sqrt(pi))) from the stored FP32 coefficients."""
    return np.maximum(0.0, 0.5 + C0 * sc.atlas[0, 11:14, 0, i].astype(np.float64))


def opacity(sc, i):
    return sigmoid(float(sc.atlas[0, 10, 0, i]))


# ------------------------------------------------------------------ the q band

Z, PX, PY = 3.0, 12, 8           # Gaussian on the optical axis at depth Z; test pixel (12, 8)


def q_scene(eps):
    """Isotropic Gaussian on the axis of a 16x16 view with principal point
    (8, 8): pixel (12, 8) has delta = (4.5, 0.5), and the log-scale is chosen
    so that q = 9 (1 + eps) there.  Returns (scene, q, alpha) by hand."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 16, 16)
    cam.cx = cam.cy = 8.0
    d2 = 4.5 ** 2 + 0.5 ** 2
    v = d2 / (9.0 * (1.0 + eps))
    ls = 0.5 * math.log((v - 0.3) * Z * Z / (cam.fx * cam.fx))
    sc = scene([dict(mu=(0.0, 0.0, Z), ls=(ls,) * 3, lo=2.0)], cam)
    s = math.exp(float(np.float32(ls)))
    q = d2 / (cam.fx * cam.fx * s * s / (Z * Z) + 0.3)
    return sc, q, min(0.99, opacity(sc, 0) * math.exp(-0.5 * q))


def pixel(fw, x, y, flips=()):
    return oracle.pixel(fw.proj[0], fw.scene.cams[0], 16, 16, fw.inst[0], fw.ranges[0], x, y, flips=flips, band=BAND)


@pytest.mark.parametrize("eps", [-INSIDE, INSIDE, -OUTSIDE, OUTSIDE])
def test_q_band(eps):
    sc, q, alpha = q_scene(eps)
    assert (abs(q - 9.0) < BAND * 9.0) == (abs(eps) == INSIDE)
    fw = oracle.Forward(sc)
    c = colour(sc, 0)
    on = q <= 9.0
    rgb, T, n, near = pixel(fw, PX, PY)
    assert near == ([0] if abs(eps) == INSIDE else [])
    # n_contrib: the pixel never stops, so it reaches the end of its one-Gaussian list
    expect = (alpha * c, 1.0 - alpha, 1) if on else (np.zeros(3), 1.0, 1)
    np.testing.assert_allclose(rgb, expect[0], rtol=1e-10, atol=1e-15)
    assert math.isclose(T, expect[1], rel_tol=1e-12) and n == expect[2]
    rgb_f, T_f, n_f, _ = pixel(fw, PX, PY, flips=[0])
    if abs(eps) == INSIDE:       # the flip takes the footprint decision the other way
        flipped = (np.zeros(3), 1.0, 1) if on else (alpha * c, 1.0 - alpha, 1)
        np.testing.assert_allclose(rgb_f, flipped[0], rtol=1e-10, atol=1e-15)
        assert math.isclose(T_f, flipped[1], rel_tol=1e-12) and n_f == flipped[2]
    else:                        # outside the band a flip changes nothing
        assert np.array_equal(rgb_f, rgb) and T_f == T and n_f == n


# ------------------------------------------------------------------ the alpha band

def alpha_scene(eps, W=16):
    """Gaussian centred on the centre of pixel (8, 8) (q = 0, alpha = o) with
    o = (1 + eps) / 255."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), W, W)
    cam.cx = cam.cy = 8.5
    return scene([dict(mu=(0.0, 0.0, 2.5), ls=(-4.0,) * 3, lo=logit((1.0 + eps) / 255.0))], cam)


@pytest.mark.parametrize("eps", [-INSIDE, INSIDE, -OUTSIDE, OUTSIDE])
def test_alpha_band(eps):
    sc = alpha_scene(eps)
    fw = oracle.Forward(sc)
    o = opacity(sc, 0)
    assert (abs(o - 1 / 255) < BAND / 255) == (abs(eps) == INSIDE)
    c = colour(sc, 0)
    on = o >= 1.0 / 255.0
    rgb, T, n, near = pixel(fw, 8, 8)
    assert near == ([0] if abs(eps) == INSIDE else [])
    expect = (o * c, 1.0 - o, 1) if on else (np.zeros(3), 1.0, 1)
    np.testing.assert_allclose(rgb, expect[0], rtol=1e-12, atol=1e-15)
    assert math.isclose(T, expect[1], rel_tol=1e-12) and n == expect[2]
    rgb_f, T_f, n_f, _ = pixel(fw, 8, 8, flips=[0])
    if abs(eps) == INSIDE:
        flipped = (np.zeros(3), 1.0, 1) if on else (o * c, 1.0 - o, 1)
        np.testing.assert_allclose(rgb_f, flipped[0], rtol=1e-12, atol=1e-15)
        assert math.isclose(T_f, flipped[1], rel_tol=1e-12) and n_f == flipped[2]
    else:
        assert np.array_equal(rgb_f, rgb) and T_f == T and n_f == n


# ------------------------------------------------------------------ the termination band

O1, O2 = 0.9, 0.95
RGB = ((0.9, 0.1, 0.4), (0.2, 0.8, 0.5), (0.3, 0.6, 0.9))


def stack_scene(eps):
    """Three Gaussians centred on pixel (8, 8) at depths 2, 3, 4 with
    opacities 0.9, 0.95 and o3 such that T (1 - o3) = 1e-4 (1 + eps) after
    the first two.  Returns (scene, (a1, a2, a3), T2, T3') by hand."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 16, 16)
    cam.cx = cam.cy = 8.5
    a1 = sigmoid(float(np.float32(logit(O1))))
    a2 = sigmoid(float(np.float32(logit(O2))))
    T2 = (1.0 * (1.0 - a1)) * (1.0 - a2)
    o3 = 1.0 - 1e-4 * (1.0 + eps) / T2
    gs = [dict(mu=(0.0, 0.0, 2.0), ls=(-4.0,) * 3, lo=logit(O1), rgb=RGB[0]),
          dict(mu=(0.0, 0.0, 3.0), ls=(-4.0,) * 3, lo=logit(O2), rgb=RGB[1]),
          dict(mu=(0.0, 0.0, 4.0), ls=(-4.0,) * 3, lo=logit(o3), rgb=RGB[2])]
    sc = scene(gs, cam)
    a3 = opacity(sc, 2)
    return sc, (a1, a2, a3), T2, T2 * (1.0 - a3)


def stack_value(sc, a, k):
    """Colour and T after compositing the first k of the stack (bg = 0)."""
    C, T = np.zeros(3), 1.0
    for i in range(k):
        C = C + T * a[i] * colour(sc, i)
        T = T * (1.0 - a[i])
    return C, T


@pytest.mark.parametrize("eps", [-INSIDE, INSIDE, -OUTSIDE, OUTSIDE])
def test_termination_band(eps):
    sc, a, T2, T3 = stack_scene(eps)
    assert (abs(T3 - 1e-4) < BAND * 1e-4) == (abs(eps) == INSIDE)
    fw = oracle.Forward(sc)
    stop = T3 < 1e-4
    rgb, T, n, near = pixel(fw, 8, 8)
    assert near == ([2] if abs(eps) == INSIDE else [])
    C, Te = stack_value(sc, a, 2 if stop else 3)
    np.testing.assert_allclose(rgb, C, rtol=1e-12)
    assert math.isclose(T, Te, rel_tol=1e-12) and n == (2 if stop else 3)
    rgb_f, T_f, n_f, _ = pixel(fw, 8, 8, flips=[2])
    if abs(eps) == INSIDE:
        C, Te = stack_value(sc, a, 3 if stop else 2)
        np.testing.assert_allclose(rgb_f, C, rtol=1e-12)
        assert math.isclose(T_f, Te, rel_tol=1e-12) and n_f == (3 if stop else 2)
    else:
        assert np.array_equal(rgb_f, rgb) and T_f == T and n_f == n


def test_two_near_decisions_flip_together():
    """Pixel (12, 8): a front Gaussian just outside its footprint (q = 9 (1 + 3e-5))
    and a back one centred there with alpha just under 1/255.  Both decisions
    are near; flipping both composites both, flipping one composites that one."""
    cam = synth.pinhole(np.eye(3), np.zeros(3), 16, 16)
    cam.cx = cam.cy = 8.0
    sc1, q, a1 = q_scene(INSIDE)
    z2 = 5.0
    mu2 = ((PX + 0.5 - 8.0) * z2 / cam.fx, (PY + 0.5 - 8.0) * z2 / cam.fy, z2)
    g1 = dict(mu=(0.0, 0.0, Z), ls=tuple(sc1.atlas[0, 3:6, 0, 0]), lo=2.0, rgb=(0.9, 0.3, 0.1))
    g2 = dict(mu=mu2, ls=(-4.0,) * 3, lo=logit((1.0 - INSIDE) / 255.0), rgb=(0.1, 0.5, 0.8))
    sc = scene([g1, g2], cam)
    fw = oracle.Forward(sc)
    c1, c2 = colour(sc, 0), colour(sc, 1)
    # the back Gaussian's mean is the pixel centre up to the FP32 rounding of its
    # position, so q ~ 1e-10 there and alpha = o to well within the tolerance below
    d = np.array([PX + 0.5, PY + 0.5]) - fw.proj[0]["mean"][1]
    assert np.abs(d).max() < 1e-5
    a2 = opacity(sc, 1)
    # nothing stops the pixel, so n_contrib is its list length (2) under every flip set
    rgb, T, n, near = pixel(fw, PX, PY)
    assert near == [0, 1] and n == 2 and np.all(rgb == 0.0) and T == 1.0
    rgb, T, n, _ = pixel(fw, PX, PY, flips=[0, 1])
    np.testing.assert_allclose(rgb, a1 * c1 + (1 - a1) * a2 * c2, rtol=1e-6)
    assert n == 2
    rgb, T, n, _ = pixel(fw, PX, PY, flips=[1])
    np.testing.assert_allclose(rgb, a2 * c2, rtol=1e-6)
    assert n == 2
    rgb, T, n, _ = pixel(fw, PX, PY, flips=[0])
    np.testing.assert_allclose(rgb, a1 * c1, rtol=1e-10)
    assert n == 2


# ------------------------------------------------------------------ adjoint under flips

def one_pixel_cotangent(cam, x, y, ch):
    G = np.zeros((3, cam.height, cam.width))
    G[ch, y, x] = 1.0
    return G


def grad2d(fw, G, flips=None):
    return oracle.backward_view(fw.proj[0], fw.scene.cams[0], 16, 16, fw.inst[0], fw.ranges[0], G, flips=flips,
                                band=BAND)


def fd_pixel(fw, x, y, ch, flips, i, field, k, h):
    """Central difference of pixel (x, y) channel ch of the flipped forward walk
    in one 2D field of Gaussian i (mean, conic, opacity or colour)."""
    out = []
    for s in (+1.0, -1.0):
        pr = fw.proj[0].copy()
        if field == "opacity":
            pr[field][i] += s * h
        else:
            pr[field][i][k] += s * h
        rgb, _, _, _ = oracle.pixel(pr, fw.scene.cams[0], 16, 16, fw.inst[0], fw.ranges[0], x, y, flips=flips,
                                    band=BAND)
        out.append(rgb[ch])
    return (out[0] - out[1]) / (2 * h)


FIELDS = [("mean", 0, 0), ("mean", 1, 1), ("conic", 0, 2), ("conic", 1, 3), ("conic", 2, 4), ("opacity", 0, 5)]


@pytest.mark.parametrize("ch", [0, 1, 2])
def test_adjoint_of_a_flipped_footprint(ch):
    """q = 9 (1 + 3e-5): not composited; flipped, the pixel composites it.
    Hand derivatives with T = 1, B = bg = 0:  dc = alpha G, dalpha = G . c,
    do = dalpha e^{-q/2}, dq = -alpha/2 dalpha, d(a, b, c) = dq (dx^2, 2 dx dy, dy^2),
    dm = -2 dq [[a, b], [b, c]] (dx, dy)."""
    sc, q, alpha = q_scene(INSIDE)
    fw = oracle.Forward(sc)
    cam = sc.cams[0]
    G = one_pixel_cotangent(cam, PX, PY, ch)
    p = PY * cam.width + PX
    assert np.all(grad2d(fw, G)[0] == 0.0)           # unflipped: q > 9, nothing reaches the Gaussian
    g = grad2d(fw, G, flips={p: [0]})[0]
    c = colour(sc, 0)
    dx, dy = PX + 0.5 - 8.0, PY + 0.5 - 8.0
    v = (dx * dx + dy * dy) / q                      # Sigma2D = v I, so the conic is I / v
    a_, b_, c_ = 1.0 / v, 0.0, 1.0 / v
    dalpha = c[ch]
    dq = -0.5 * alpha * dalpha
    hand = np.zeros(9)
    hand[6 + ch] = alpha
    hand[5] = dalpha * math.exp(-0.5 * q)
    hand[2:5] = dq * np.array([dx * dx, 2 * dx * dy, dy * dy])
    hand[0] = -2.0 * dq * (a_ * dx + b_ * dy)
    hand[1] = -2.0 * dq * (b_ * dx + c_ * dy)
    np.testing.assert_allclose(g, hand, rtol=1e-9, atol=1e-18)
    # central differences of the flipped forward walk
    for field, k, j in FIELDS:
        h = 1e-6 * max(1.0, abs(float(np.atleast_1d(fw.proj[0][field][0])[k])))
        np.testing.assert_allclose(fd_pixel(fw, PX, PY, ch, [0], 0, field, k, h), g[j], rtol=1e-6, atol=1e-12)
    for k in range(3):
        fdv = fd_pixel(fw, PX, PY, ch, [0], 0, "color", k, 1e-6)
        np.testing.assert_allclose(fdv, g[6 + k], rtol=1e-6, atol=1e-12)
    # the same scene moved inside the footprint, unflipped
    sc2, _, _ = q_scene(-INSIDE)
    g2 = grad2d(oracle.Forward(sc2), G)[0]
    np.testing.assert_allclose(g, g2, rtol=1e-3)


@pytest.mark.parametrize("ch", [0, 2])
def test_adjoint_of_a_flipped_termination(ch):
    """T' = 1e-4 (1 - 3e-5): the walk stops before the third Gaussian; flipped,
    it composites it.  Hand derivatives of C = a1 c1 + (1 - a1) a2 c2 +
    (1 - a1)(1 - a2) a3 c3 (q = 0, so dL/do = dL/dalpha)."""
    sc, a, T2, T3 = stack_scene(-INSIDE)
    fw = oracle.Forward(sc)
    cam = sc.cams[0]
    G = one_pixel_cotangent(cam, 8, 8, ch)
    p = 8 * cam.width + 8
    c = [colour(sc, i)[ch] for i in range(3)]
    a1, a2, a3 = a
    g = grad2d(fw, G, flips={p: [2]})
    hand_do = [c[0] - a2 * c[1] - (1 - a2) * a3 * c[2], (1 - a1) * (c[1] - a3 * c[2]), (1 - a1) * (1 - a2) * c[2]]
    hand_dc = [a1, (1 - a1) * a2, (1 - a1) * (1 - a2) * a3]
    np.testing.assert_allclose(g[:, 5], hand_do, rtol=1e-9)
    np.testing.assert_allclose(g[:, 6 + ch], hand_dc, rtol=1e-9)
    g0 = grad2d(fw, G)                                # unflipped: the third Gaussian gets nothing
    assert np.all(g0[2] == 0.0)
    for i in range(3):
        np.testing.assert_allclose(fd_pixel(fw, 8, 8, ch, [2], i, "opacity", 0, 1e-7), g[i, 5], rtol=1e-6)
        np.testing.assert_allclose(fd_pixel(fw, 8, 8, ch, [2], i, "color", ch, 1e-6), g[i, 6 + ch], rtol=1e-6)
    sc2, _, _, _ = stack_scene(INSIDE)            # moved past the threshold, unflipped
    np.testing.assert_allclose(g, grad2d(oracle.Forward(sc2), G), rtol=1e-3, atol=1e-12)
