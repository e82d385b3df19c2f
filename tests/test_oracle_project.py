"""Pins for the oracle's fetch, SH basis and EWA projection.

Each test checks the oracle against something other than its own formulas:
closed forms of the EWA chain (Alg. 1 steps 1-4), a library rotation routine,
scipy's complex spherical harmonics, quadrature, or brute-force enumeration.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
import synth

F_128 = synth.focal_for_hfov(128)


def one_gaussian(mu, lscale, quat=(1, 0, 0, 0), lopac=0.0, sh=None, L=0):
    C = synth.n_channels(L)
    P = np.zeros((C, 1), np.float64)
    P[0:3, 0] = mu
    P[3:6, 0] = lscale
    P[6:10, 0] = quat
    P[10, 0] = lopac
    if sh is not None:
        P[11:11 + len(sh), 0] = sh
    return P


def ident_cam(w=128, h=128):
    return synth.pinhole(np.eye(3), np.zeros(3), w, h)


# ------------------------------------------------------------------ fetch

def test_fetch_invariants():
    rng = np.random.default_rng(0)
    occ = (rng.random((13, 17)) < 0.6).astype(np.uint8)
    atlas = rng.standard_normal((2, 5, 13, 17)).astype(np.float32)
    ids, params = oracle.fetch(atlas, occ)
    assert ids.size == int(occ.sum())
    assert np.array_equal(ids, np.flatnonzero(occ.reshape(-1)))
    assert np.array_equal(params, atlas.reshape(2, 5, -1)[:, :, ids].astype(np.float64))
    # scatter(gather(x)) = x on occupied texels, 0 elsewhere
    back = oracle.scatter(params, ids, None, 13, 17)
    assert np.array_equal(back, atlas * occ[None, None])
    # <gather x, y> = <x, scatter y>
    y = rng.standard_normal(params.shape)
    sy = oracle.scatter(y, ids, None, 13, 17)
    assert math.isclose(float((params * y).sum()), float((atlas.astype(np.float64) * sy).sum()), rel_tol=1e-12)


def test_scatter_freeze_mask():
    rng = np.random.default_rng(1)
    occ = np.ones((4, 4), np.uint8)
    ids = np.arange(16, dtype=np.int32)
    g = rng.standard_normal((1, 3, 16))
    dyn = (rng.random((4, 4)) < 0.5).astype(np.uint8)
    out = oracle.scatter(g, ids, dyn, 4, 4)
    assert np.array_equal(out[0].reshape(3, 16), g[0] * dyn.reshape(-1)[None])
    assert not np.any(out[0].reshape(3, 16)[:, dyn.reshape(-1) == 0])


# ------------------------------------------------------------------ SH

def real_sh_from_scipy(l, m, d):
    """Real SH (Condon-Shortley phase kept) from scipy's complex Y_l^m:
    sqrt(2) Im Y_l^{|m|} for m < 0, Y_l^0, sqrt(2) Re Y_l^m for m > 0."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m < 0:
        return math.sqrt(2.0) * Y.imag
    if m == 0:
        return Y.real
    return math.sqrt(2.0) * Y.real


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B = oracle.sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            j = l * l + l + m
            np.testing.assert_allclose(B[:, j], real_sh_from_scipy(l, m, d), rtol=0, atol=1e-12,
                                       err_msg=f"l={l} m={m}")


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi integrates degree <= 6 exactly.
    xs, ws = np.polynomial.legendre.leggauss(16)
    nphi = 32
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xs, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (ws[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    B = oracle.sh_basis(d, 3)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


# ------------------------------------------------------------------ projection closed forms

@pytest.mark.parametrize("z,sigma", [(2.0, 0.02), (3.0, 0.05), (7.5, 0.11)])
def test_on_axis_isotropic(z, sigma):
    cam = ident_cam()
    P = one_gaussian((0.0, 0.0, z), [math.log(sigma)] * 3)
    pr = oracle.project(P, 0, cam, 16, 16)[0]
    v = F_128 ** 2 * sigma ** 2 / z ** 2 + 0.3
    assert pr["valid"] == 1
    np.testing.assert_allclose(pr["mean"], [64.0, 64.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(pr["cov2d"], [v, 0.0, v], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(pr["conic"], [1 / v, 0.0, 1 / v], rtol=1e-12, atol=1e-15)
    assert pr["radius"] == math.ceil(3 * math.sqrt(v))
    r = pr["radius"]
    assert list(pr["rect"]) == [max(0, (64 - r) // 16), max(0, (64 - r) // 16), min(7, (64 + r) // 16),
                                min(7, (64 + r) // 16)]
    assert pr["key"] == np.float32(z).view(np.uint32)


def test_off_axis_isotropic_JJt():
    cam = synth.pinhole(np.eye(3), np.zeros(3), 160, 120)
    f = cam.fx
    rng = np.random.default_rng(3)
    for _ in range(20):
        x, y, z = rng.uniform(-0.8, 0.8), rng.uniform(-0.6, 0.6), rng.uniform(2.0, 5.0)
        sigma = rng.uniform(0.005, 0.05)
        pr = oracle.project(one_gaussian((x, y, z), [math.log(sigma)] * 3), 0, cam, 16, 16)[0]
        JJt = np.array([[f * f / z ** 2 + f * f * x * x / z ** 4, f * f * x * y / z ** 4],
                        [f * f * x * y / z ** 4, f * f / z ** 2 + f * f * y * y / z ** 4]])
        S = sigma ** 2 * JJt + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(pr["mean"], [f * x / z + cam.cx, f * y / z + cam.cy], rtol=1e-13)
        np.testing.assert_allclose(pr["det"], np.linalg.det(S), rtol=1e-11)


def test_anisotropic_on_axis_matches_rotation_library():
    """Sigma = R(q) diag(s^2) R(q)^T with q = (w, x, y, z); on the optical axis of
    an identity camera Sigma2D = (f/z)^2 Sigma[:2, :2] + 0.3 I."""
    cam = ident_cam()
    rng = np.random.default_rng(4)
    for _ in range(20):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        ls = rng.normal(-3.5, 0.5, 3)
        z = rng.uniform(2, 4)
        pr = oracle.project(one_gaussian((0, 0, z), ls, q), 0, cam, 16, 16)[0]
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = R @ np.diag(np.exp(2 * ls)) @ R.T
        np.testing.assert_allclose(np.linalg.eigvalsh(Sig), np.sort(np.exp(2 * ls)), rtol=1e-10)
        S2 = (F_128 / z) ** 2 * Sig[:2, :2] + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-10, atol=1e-13)


def test_quaternion_scale_invariance():
    """The stored quaternion need not be unit: q and 3.7 q give the same Gaussian."""
    cam = ident_cam()
    q = np.array([0.3, -0.5, 0.2, 0.7])
    a = oracle.project(one_gaussian((0.1, 0.2, 3.0), (-3.3, -3.0, -3.6), q), 0, cam, 16, 16)[0]
    b = oracle.project(one_gaussian((0.1, 0.2, 3.0), (-3.3, -3.0, -3.6), 3.7 * q), 0, cam, 16, 16)[0]
    np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-12)


def test_rotation_about_optical_axis_rotates_cov2d():
    cam = ident_cam()
    q0 = np.array([0.9, 0.1, -0.3, 0.2])
    q0 /= np.linalg.norm(q0)
    ls = (-3.0, -3.8, -3.4)
    base = oracle.project(one_gaussian((0, 0, 3.0), ls, q0), 0, cam, 16, 16)[0]
    S0 = np.array([[base["cov2d"][0], base["cov2d"][1]], [base["cov2d"][1], base["cov2d"][2]]]) - 0.3 * np.eye(2)
    for th in (0.3, 1.1, 2.5):
        rz = Rotation.from_euler("z", th)
        qr = (rz * Rotation.from_quat([q0[1], q0[2], q0[3], q0[0]])).as_quat()
        pr = oracle.project(one_gaussian((0, 0, 3.0), ls, (qr[3], qr[0], qr[1], qr[2])), 0, cam, 16, 16)[0]
        c, s = math.cos(th), math.sin(th)
        R2 = np.array([[c, -s], [s, c]])
        S = R2 @ S0 @ R2.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-10, atol=1e-12)


def test_look_at_target_projects_to_principal_point():
    for cam in synth.ring_cameras(8, 4.0, 512, 384) + synth.fibonacci_cameras(13, 4.0, 320, 240):
        pr = oracle.project(one_gaussian((0, 0, 0), (-4, -4, -4)), 0, cam, 16, 16)[0]
        np.testing.assert_allclose(pr["mean"], [cam.cx, cam.cy], atol=1e-9)
        assert abs(pr["z"] - 4.0) < 1e-12


def test_culling_near_plane_and_behind():
    cam = ident_cam()
    for z in (-1.0, 0.0, 0.1, 0.2):
        assert oracle.project(one_gaussian((0, 0, z), (-3, -3, -3)), 0, cam, 16, 16)[0]["valid"] == 0
    assert oracle.project(one_gaussian((0, 0, 0.2001), (-3, -3, -3)), 0, cam, 16, 16)[0]["valid"] == 1
    # fully off-screen: empty rectangle
    assert oracle.project(one_gaussian((5.0, 0, 2.0), (-5, -5, -5)), 0, cam, 16, 16)[0]["valid"] == 0


def test_degree0_colour_and_clamp():
    cam = ident_cam()
    C0 = 0.5 / math.sqrt(math.pi)
    for k in (-3.0, -1.0, 0.0, 0.4, 2.0):
        pr = oracle.project(one_gaussian((0, 0, 3), (-3,) * 3, sh=[k, 2 * k, -k]), 0, cam, 16, 16)[0]
        raw = 0.5 + C0 * np.array([k, 2 * k, -k])
        np.testing.assert_allclose(pr["color_raw"], raw, rtol=1e-14)
        np.testing.assert_allclose(pr["color"], np.maximum(raw, 0), rtol=1e-14)


def test_sigmoid_opacity():
    cam = ident_cam()
    for lo in (-4.0, 0.0, 1.5):
        pr = oracle.project(one_gaussian((0, 0, 3), (-3,) * 3, lopac=lo), 0, cam, 16, 16)[0]
        assert math.isclose(pr["opacity"], 1 / (1 + math.exp(-lo)), rel_tol=1e-15)


def test_rect_covers_every_pixel_inside_the_ellipse():
    """Brute force over pixels: any pixel centre with q <= 9 lies in a tile of the rectangle."""
    sc = synth.random_scene(side=10, sh_degree=0, views=3, width=96, height=80, seed=5, lscale=(-2.5, 0.6))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    for tw, th in ((16, 16), (8, 32), (32, 8)):
        for cam in sc.cams:
            pr = oracle.project(params[0], 0, cam, tw, th)
            ys, xs = np.mgrid[0:cam.height, 0:cam.width]
            for g in pr[pr["valid"] == 1][:40]:
                dx = xs + 0.5 - g["mean"][0]
                dy = ys + 0.5 - g["mean"][1]
                a, b, c = g["conic"]
                inside = a * dx * dx + 2 * b * dx * dy + c * dy * dy <= 9.0
                tx, ty = xs[inside] // tw, ys[inside] // th
                assert np.all((tx >= g["rect"][0]) & (tx <= g["rect"][2]))
                assert np.all((ty >= g["rect"][1]) & (ty <= g["rect"][3]))


def in_rect(g, tx, ty):
    r = g["rect"]
    return bool(r[0] <= tx <= r[2] and r[1] <= ty <= r[3])


def test_visibility_at_the_image_border():
    """visible: past the z / det culls and some pixel of the image within r of
    the mean on both axes.  An isotropic Gaussian on a shifted principal point
    is moved across each border: it is visible exactly while m + r >= 0 on the
    left (top) and m - r < W (H) on the right (bottom), hand-evaluated from
    the radius of the on-axis closed form."""
    z, ls = 3.0, -3.5
    s = math.exp(float(np.float32(ls)))
    for W, H in ((40, 24), (37, 29)):
        cam = ident_cam(W, H)
        r = math.ceil(3 * math.sqrt(cam.fx ** 2 * s * s / (z * z) + 0.3))
        for cx, cy, expect in ((-r + 0.25, H / 2, True), (-r - 0.25, H / 2, False),
                               (W + r - 0.25, H / 2, True), (W + r + 0.25, H / 2, False),
                               (W / 2, -r + 0.25, True), (W / 2, -r - 0.25, False),
                               (W / 2, H + r - 0.25, True), (W / 2, H + r + 0.25, False)):
            cam.cx, cam.cy = cx, cy
            for tw, th in ((16, 16), (8, 32), (32, 8)):
                g = oracle.project(one_gaussian((0, 0, z), (ls,) * 3), 0, cam, tw, th)[0]
                assert g["radius"] == r
                assert bool(g["visible"]) == expect, (W, H, cx, cy, tw, th)
                if expect:
                    assert g["valid"] == 1   # a visible Gaussian is always listed
    # behind the near plane: neither listed nor visible
    g = oracle.project(one_gaussian((0, 0, 0.1), (ls,) * 3), 0, ident_cam(), 16, 16)[0]
    assert g["valid"] == 0 and g["visible"] == 0


def test_visibility_independent_of_tile_shape():
    """Ragged views (width and height not multiples of any tile side): the
    visible flags are the same for every tile shape, every visible Gaussian
    is listed, and Gaussians listed only because a ragged tile reaches past
    the image edge are not visible and have no pixel with q <= 9."""
    sc = synth.random_scene(side=14, sh_degree=0, views=3, width=85, height=43, seed=21, lscale=(-2.6, 0.6))
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    n_edge = 0
    for cam in sc.cams:
        cam.cx, cam.cy = cam.width, cam.height    # scene centred on the bottom-right corner
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        ref = None
        for tw, th in ((16, 16), (8, 32), (32, 8)):
            pr = oracle.project(params[0], 0, cam, tw, th)
            vis = pr["visible"].copy()
            if ref is None:
                ref = vis
            assert np.array_equal(vis, ref)
            assert np.all(pr["valid"][vis == 1] == 1)
            for g in pr[(pr["valid"] == 1) & (pr["visible"] == 0)]:
                n_edge += 1
                dx, dy = xs + 0.5 - g["mean"][0], ys + 0.5 - g["mean"][1]
                a, b, c = g["conic"]
                assert not np.any(a * dx * dx + 2 * b * dx * dy + c * dy * dy <= 9.0)
        assert 0 < ref.sum() < len(ref)
    assert n_edge > 0, "the scene must list Gaussians that are not visible"


def test_bin_sort_matches_brute_force_enumeration():
    sc = synth.random_scene(side=12, sh_degree=0, views=2, width=100, height=70, seed=6)
    ids, params = oracle.fetch(sc.atlas, sc.occupancy)
    for tw, th in ((16, 16), (8, 32)):
        for cam in sc.cams:
            pr = oracle.project(params[0], 0, cam, tw, th)
            inst, ranges = oracle.bin_sort(pr, cam, tw, th)
            TX, TY = oracle.tiles_of(cam, tw, th)
            brute = []
            for t in range(TX * TY):
                tx, ty = t % TX, t // TX
                for i in range(pr.shape[0]):
                    if pr[i]["valid"] and in_rect(pr[i], tx, ty):
                        brute.append((t, int(pr[i]["key"]), i))
            brute.sort()
            got = [(int(a), int(b), int(c)) for a, b, c in zip(inst["tile"], inst["key"], inst["id"])]
            assert got == brute
            v = pr[pr["valid"] == 1]
            area = (v["rect"][:, 2] - v["rect"][:, 0] + 1) * (v["rect"][:, 3] - v["rect"][:, 1] + 1)
            assert np.array_equal(v["n_tiles"], area)
            assert len(inst) == int(area.sum())
            assert np.all(pr[pr["valid"] == 0]["n_tiles"] == 0)
            # ranges partition [0, I)
            nonempty = ranges[ranges[:, 1] > ranges[:, 0]]
            assert nonempty[0, 0] == 0 and nonempty[-1, 1] == len(inst)
            assert np.all(nonempty[1:, 0] == nonempty[:-1, 1])
