"""FP64 CPU oracle for the PackUV-GS splatting path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and the
two share no code: the oracle's arithmetic lives in ``oracle.c`` (plain C,
FP64, built with ``-ffp-contract=off -fno-fast-math``); this module only
marshals numpy arrays in and out of it.

Parity status of each function (what pins it; see ``tests/test_oracle_*.py``):
  fetch             -- invariants: N = popcount, row-major ids, gather/scatter identity.
  project           -- closed forms: on-axis isotropic Sigma2D and radius, off-axis
                       J J^T, eig(Sigma) = s^2, look-at target -> principal point,
                       rotation about the optical axis; SH basis against scipy's
                       complex SH and quadrature orthonormality.
  bin_sort          -- brute-force rectangle membership + textbook sort; every tile of
                       the rectangle is listed (no culling inside the rectangle).
  render            -- single Gaussian, stacked-Gaussian transmittance product,
                       two-Gaussian closed form; tiled == brute force bitwise (brute
                       force walks every Gaussian past the z / det culls, no rectangles).
  pixel (near / flips) -- one-pixel scenes with q, alpha and T' just inside and just
                       outside each guard band: the near list, and the value a flip gives,
                       against hand-evaluated compositing.
  backward          -- two-Gaussian closed-form derivatives; central finite
                       differences of the forward with frozen decisions; under
                       flips, against hand-evaluated derivatives and against the
                       unflipped adjoint of the scene moved across the threshold.
  visible           -- hand cases at the image border; independence of the tile shape.
  loss_l1, adam     -- textbook closed forms.
  uv_prune          -- axis directions and the theta = pi / phi = pi edges of the UV equation;
                       numpy brute force (arctan2, arccos, lexsort) for the pixels and ranks.
  ssim              -- SSIM(x, x) = 1 with zero gradient; constant planes against the closed
                       form (2ab + C1)/(a^2 + b^2 + C1) in the interior; window statistics
                       against scipy.ndimage.correlate; symmetry; FD of the gradient.
  regularisers      -- hand-evaluated hinge and o (1 - o) on chosen values; FD of both.
  flow_mask         -- on-axis isotropic disc closed form (pixels just inside / outside
                       3 sigma), brute force over every pixel of the image, OR across
                       cameras, empty and full masks.
  fake_quant        -- unit-step grid against numpy's rint, brute-force nearest level,
                       endpoints, monotonicity, untouched texels and channels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PROJ_DTYPE = np.dtype([
    ("valid", "<i4"), ("radius", "<i4"), ("rect", "<i4", (4,)), ("key", "<u4"), ("pad", "<u4"),
    ("z", "<f8"), ("mean", "<f8", (2,)), ("cov2d", "<f8", (3,)), ("det", "<f8"),
    ("conic", "<f8", (3,)), ("opacity", "<f8"), ("color", "<f8", (3,)), ("color_raw", "<f8", (3,)),
    ("visible", "<i4"), ("pad2", "<i4"), ("n_tiles", "<i8"),
])
INST_DTYPE = np.dtype([("tile", "<i8"), ("key", "<u4"), ("id", "<i4")])
CAM_DTYPE = np.dtype([
    ("R", "<f8", (9,)), ("t", "<f8", (3,)), ("fx", "<f8"), ("fy", "<f8"), ("cx", "<f8"), ("cy", "<f8"),
    ("width", "<i4"), ("height", "<i4"), ("frame", "<i4"), ("reserved", "<i4"),
])
assert PROJ_DTYPE.itemsize == 184 and CAM_DTYPE.itemsize == 144 and INST_DTYPE.itemsize == 16

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        p, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "or_sh_basis": (None, [p, i64, i32, p]),
            "or_fetch": (i64, [p, p, i32, i32, i32, i32, p, p]),
            "or_project": (None, [p, i64, i32, i32, p, i32, i32, p]),
            "or_count_instances": (i64, [p, i64]),
            "or_bin_sort": (None, [p, i64, p, i32, i32, p, p]),
            "or_render": (None, [p, p, i32, i32, p, p, p, p, p, p, p]),
            "or_render_brute": (None, [p, i64, p, p, p, p, p]),
            "or_pixel": (i32, [p, p, i32, i32, p, p, p, i32, i32, p, i32, f64, p, i32, p, p, p]),
            "or_loss_l1": (f64, [p, p, i64, p]),
            "or_backward_view": (None, [p, i64, p, i32, i32, p, p, p, p, p, p, i32, f64, p]),
            "or_project_backward": (None, [p, i64, i32, p, p, p, p]),
            "or_scatter": (None, [p, p, p, i32, i32, i32, i32, i64, p]),
            "or_fd_frozen": (f64, [p, i64, i32, i32, p, i32, i32, p, p, p, p, p, i64, i32, f64]),
            "or_adam": (None, [p, p, p, p, p, i64, f64, f64, f64, f64, i32]),
            "or_fake_quant": (None, [p, p, i32, i32, i32, i32, p, p, p, p]),
            "or_flow_mask": (None, [p, i64, i32, p, p, p]),
            "or_ssim": (f64, [p, p, i32, i32, p, p]),
            "or_uv_prune": (None, [p, i64, i32, i32, i32, p, p, p, p]),
            "or_regularisers": (i64, [p, i32, i32, i64, p, f64, f64, f64, p, p]),
            "or_num_threads": (i32, []),
            "or_set_num_threads": (None, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def cam_record(cam) -> np.ndarray:
    r = np.zeros(1, CAM_DTYPE)
    r["R"][0] = np.asarray(cam.R, np.float64).reshape(9)
    r["t"][0] = np.asarray(cam.t, np.float64).reshape(3)
    r["fx"], r["fy"], r["cx"], r["cy"] = cam.fx, cam.fy, cam.cx, cam.cy
    r["width"], r["height"], r["frame"] = cam.width, cam.height, cam.frame
    return r


def tiles_of(cam, tw, th):
    return (cam.width + tw - 1) // tw, (cam.height + th - 1) // th


# --------------------------------------------------------------------------- stages

def sh_basis(dirs: np.ndarray, L: int) -> np.ndarray:
    d = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((d.shape[0], (L + 1) ** 2), np.float64)
    lib().or_sh_basis(_p(d), d.shape[0], L, _p(out))
    return out


def fetch(atlas: np.ndarray, occ: np.ndarray):
    atlas = np.ascontiguousarray(atlas, np.float32)
    occ = np.ascontiguousarray(occ, np.uint8)
    F, Cc, H, W = atlas.shape
    n = int(np.count_nonzero(occ))
    ids = np.zeros(max(n, 1), np.int32)
    params = np.zeros((F, Cc, max(n, 1)), np.float64)
    got = lib().or_fetch(_p(atlas), _p(occ), F, Cc, H, W, _p(ids), _p(params))
    assert got == n
    return ids[:n], np.ascontiguousarray(params[:, :, :n])


def uv_prune(params_f: np.ndarray, M: int, Nv: int, K: int, expected=None):
    """(uv, rank, keep) of one frame's Gaussians (C, N) on an M x Nv UV map."""
    P = np.ascontiguousarray(params_f, np.float64)
    Cc, N = P.shape
    uv = np.zeros(max(N, 1), np.int32)
    rank = np.zeros(max(N, 1), np.int32)
    keep = np.zeros(max(N, 1), np.uint8)
    e = None if expected is None else np.ascontiguousarray(expected, np.int32)
    lib().or_uv_prune(_p(P), N, int(M), int(Nv), int(K), _p(e) if e is not None else None, _p(uv), _p(rank),
                      _p(keep))
    return uv[:N], rank[:N], keep[:N]


def ssim(x: np.ndarray, y: np.ndarray, grad: bool = False, smap: bool = False):
    """Sum over an (H, W) plane of the SSIM map of x against y, and (if grad)
    its gradient with respect to x, (if smap) the map itself."""
    xx = np.ascontiguousarray(x, np.float64)
    yy = np.ascontiguousarray(y, np.float64)
    H, W = xx.shape
    g = np.zeros((H, W), np.float64) if grad else None
    m = np.zeros((H, W), np.float64) if smap else None
    tot = lib().or_ssim(_p(xx), _p(yy), H, W, _p(g) if grad else None, _p(m) if smap else None)
    out = (tot,) + ((g,) if grad else ()) + ((m,) if smap else ())
    return out if len(out) > 1 else tot


def regularisers(params: np.ndarray, s_max: float, w_scale: float = 1.0, w_opacity: float = 1.0, dyn=None):
    """(L_scale, L_opacity, gradient (F, C, N) of w_scale L_scale + w_opacity
    L_opacity, number of Gaussians averaged) over params (F, C, N)."""
    P = np.ascontiguousarray(params, np.float64)
    F, Cc, N = P.shape
    d = None if dyn is None else np.ascontiguousarray(dyn, np.uint8).reshape(F * N)
    g = np.zeros_like(P)
    out = np.zeros(2, np.float64)
    n = lib().or_regularisers(_p(P), F, Cc, N, _p(d) if d is not None else None, float(s_max), float(w_scale),
                              float(w_opacity), _p(g), _p(out))
    return float(out[0]), float(out[1]), g, int(n)


def photo_loss(images: dict, targets: dict, lam_ssim: float):
    """(1 - lam) mean |I - T| + lam (1 - mean SSIM) over every view, pixel and
    channel, and its cotangents dL/dI per view (3, H, W)."""
    views = list(images)
    n = sum(images[v].size for v in views)
    l1 = sum(float(np.abs(np.asarray(images[v], np.float64) - targets[v]).sum()) for v in views)
    s_sum, G = 0.0, {}
    for v in views:
        I = np.asarray(images[v], np.float64)
        T = np.asarray(targets[v], np.float64)
        g = np.zeros_like(I)
        for ch in range(I.shape[0]):
            s, gs = ssim(I[ch], T[ch], grad=True)
            s_sum += s
            g[ch] = -lam_ssim * gs / n
        G[v] = g + (1.0 - lam_ssim) * np.sign(I - T) / n
    L = (1.0 - lam_ssim) * l1 / n + lam_ssim * (1.0 - s_sum / n)
    return L, G


def flow_mask(params_f: np.ndarray, sh_degree: int, cam, mask: np.ndarray, D: np.ndarray | None = None):
    """Dynamic labels (N,) uint8 of one frame's Gaussians for one camera's flow
    mask (H, W), OR-ed into D when given."""
    P = np.ascontiguousarray(params_f, np.float64)
    Cc, N = P.shape
    m = np.ascontiguousarray(mask, np.uint8)
    assert m.shape == (cam.height, cam.width)
    out = np.zeros(N, np.uint8) if D is None else D
    assert out.dtype == np.uint8 and out.flags.c_contiguous
    lib().or_flow_mask(_p(P), N, sh_degree, _p(cam_record(cam)), _p(m), _p(out))
    return out


def fake_quant(atlas: np.ndarray, occ: np.ndarray, bits):
    """LPO proxy of an atlas (F, C, H, W): returns (proxy atlas, range (C, 2), codes uint16)."""
    atlas = np.ascontiguousarray(atlas, np.float32)
    occ = np.ascontiguousarray(occ, np.uint8)
    F, Cc, H, W = atlas.shape
    b = np.ascontiguousarray(bits, np.int32)
    assert b.shape == (Cc,)
    out = np.empty_like(atlas)
    rng = np.zeros((Cc, 2), np.float32)
    codes = np.zeros(atlas.shape, np.uint16)
    lib().or_fake_quant(_p(atlas), _p(occ), F, Cc, H, W, _p(b), _p(rng), _p(out), _p(codes))
    return out, rng, codes


def project(params_f: np.ndarray, sh_degree: int, cam, tw: int, th: int) -> np.ndarray:
    P = np.ascontiguousarray(params_f, np.float64)
    Cc, N = P.shape
    out = np.zeros(N, PROJ_DTYPE)
    cr = cam_record(cam)
    lib().or_project(_p(P), N, Cc, sh_degree, _p(cr), tw, th, _p(out))
    return out


def bin_sort(proj: np.ndarray, cam, tw: int, th: int):
    N = proj.shape[0]
    I = int(lib().or_count_instances(_p(proj), N))
    inst = np.zeros(max(I, 1), INST_DTYPE)
    TX, TY = tiles_of(cam, tw, th)
    ranges = np.zeros((TX * TY, 2), np.int64)
    cr = cam_record(cam)
    lib().or_bin_sort(_p(proj), N, _p(cr), tw, th, _p(inst), _p(ranges))
    return inst[:I], ranges


def render(proj, cam, tw, th, inst, ranges, bg=(0.0, 0.0, 0.0)):
    H, W = cam.height, cam.width
    ids = np.ascontiguousarray(inst["id"], np.int32) if len(inst) else np.zeros(1, np.int32)
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    n = np.zeros((H, W), np.int32)
    counts = np.zeros(2, np.int64)
    bgv = np.asarray(bg, np.float64)
    cr = cam_record(cam)
    lib().or_render(_p(proj), _p(cr), tw, th, _p(ids), _p(np.ascontiguousarray(ranges)), _p(bgv),
                    _p(img), _p(T), _p(n), _p(counts))
    return img, T, n, counts


def render_brute(proj, cam, bg=(0.0, 0.0, 0.0)):
    H, W = cam.height, cam.width
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    n = np.zeros((H, W), np.int32)
    bgv = np.asarray(bg, np.float64)
    cr = cam_record(cam)
    lib().or_render_brute(_p(proj), proj.shape[0], _p(cr), _p(bgv), _p(img), _p(T), _p(n))
    return img, T, n


def pixel(proj, cam, tw, th, inst, ranges, x, y, flips=(), band=1e-4, bg=(0.0, 0.0, 0.0), max_near=64):
    ids = np.ascontiguousarray(inst["id"], np.int32) if len(inst) else np.zeros(1, np.int32)
    fl = np.asarray(list(flips) or [-1], np.int32)
    near = np.zeros(max_near, np.int32)
    rgb = np.zeros(3, np.float64)
    T = np.zeros(1, np.float64)
    n = np.zeros(1, np.int32)
    bgv = np.asarray(bg, np.float64)
    cr = cam_record(cam)
    nn = lib().or_pixel(_p(proj), _p(cr), tw, th, _p(ids), _p(np.ascontiguousarray(ranges)), _p(bgv),
                        int(x), int(y), _p(fl), len(flips), band, _p(near), max_near, _p(rgb), _p(T), _p(n))
    return rgb, float(T[0]), int(n[0]), [int(v) for v in near[:min(nn, max_near)]]


def loss_l1(img: np.ndarray, target: np.ndarray, n_total: int | None = None):
    """L = mean |img - target|; G = sign(img - target) / n (sign(0) = 0)."""
    a = np.ascontiguousarray(img, np.float64).reshape(-1)
    b = np.ascontiguousarray(target, np.float64).reshape(-1)
    G = np.zeros_like(a)
    L = lib().or_loss_l1(_p(a), _p(b), a.size, _p(G))
    return float(L), G.reshape(np.shape(img))


def backward_view(proj, cam, tw, th, inst, ranges, G, bg=(0.0, 0.0, 0.0), flips=None, band=1e-4):
    """Per-Gaussian 2D gradients (N, 9): dm_x, dm_y, da, db, dc, do, dr, dg, db_col.
    ``flips`` maps a pixel index (y * W + x) to up to two list positions."""
    N = proj.shape[0]
    ids = np.ascontiguousarray(inst["id"], np.int32) if len(inst) else np.zeros(1, np.int32)
    Gc = np.ascontiguousarray(G, np.float64)
    flips = flips or {}
    fpix = np.asarray(list(flips.keys()) or [-1], np.int32)
    fpos = np.full((max(len(flips), 1), 2), -1, np.int32)
    for j, v in enumerate(flips.values()):
        v = list(v)[:2]
        fpos[j, :len(v)] = v
    out = np.zeros((max(N, 1), 9), np.float64)
    bgv = np.asarray(bg, np.float64)
    cr = cam_record(cam)
    lib().or_backward_view(_p(proj), N, _p(cr), tw, th, _p(ids), _p(np.ascontiguousarray(ranges)), _p(bgv),
                           _p(Gc), _p(fpix), _p(fpos), len(flips), band, _p(out))
    return out[:N]


def project_backward(params_f, sh_degree, cam, proj, grad2d, gP):
    P = np.ascontiguousarray(params_f, np.float64)
    g2 = np.ascontiguousarray(grad2d, np.float64)
    assert gP.flags.c_contiguous and gP.dtype == np.float64
    cr = cam_record(cam)
    lib().or_project_backward(_p(P), P.shape[1], sh_degree, _p(cr), _p(proj), _p(g2), _p(gP))


def scatter(gP: np.ndarray, ids: np.ndarray, dyn, H: int, W: int) -> np.ndarray:
    F, Cc, N = gP.shape
    out = np.zeros((F, Cc, H, W), np.float64)
    d = None if dyn is None else np.ascontiguousarray(dyn, np.uint8)
    lib().or_scatter(_p(np.ascontiguousarray(gP)), _p(np.ascontiguousarray(ids, np.int32)), _p(d), F, Cc, H, W,
                     N, _p(out))
    return out


def fd_frozen(params_f, sh_degree, cam, tw, th, proj, inst, ranges, G, i, ch, h, bg=(0.0, 0.0, 0.0)):
    P = np.ascontiguousarray(params_f, np.float64)
    ids = np.ascontiguousarray(inst["id"], np.int32) if len(inst) else np.zeros(1, np.int32)
    bgv = np.asarray(bg, np.float64)
    cr = cam_record(cam)
    return float(lib().or_fd_frozen(_p(P), P.shape[1], P.shape[0], sh_degree, _p(cr), tw, th, _p(proj), _p(ids),
                                     _p(np.ascontiguousarray(ranges)), _p(bgv),
                                     _p(np.ascontiguousarray(G, np.float64)), int(i), int(ch), float(h)))


def adam(p, g, m, v, visible, lr, b1, b2, eps, t):
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, np.float64)
    vis = np.ascontiguousarray(visible, np.uint8)
    lib().or_adam(_p(p), _p(g), _p(m), _p(v), _p(vis), p.size, lr, b1, b2, eps, int(t))


# --------------------------------------------------------------------------- whole scene

class Forward:
    """Oracle forward pass over every view of a scene."""

    def __init__(self, scene, views=None, bg=None, counts=False, quant_bits=None):
        """quant_bits: per-channel bit widths of the LPO proxy (None: no
        quantisation).  With a proxy the whole pass runs on it, and the
        straight-through texel gradient is the gradient at the proxy."""
        self.scene = scene
        tl = scene.tiling
        self.tw, self.th = tl.tile_w, tl.tile_h
        self.bg = tuple(scene.bg if bg is None else bg)
        atlas = scene.atlas
        self.quant = None
        if quant_bits is not None:
            atlas, rng, codes = fake_quant(scene.atlas, scene.occupancy, quant_bits)
            self.quant = (rng, codes)
        self.ids, self.params = fetch(atlas, scene.occupancy)
        self.views = list(range(len(scene.cams))) if views is None else list(views)
        self.proj, self.inst, self.ranges = {}, {}, {}
        self.image, self.T, self.n, self.counts = {}, {}, {}, {}
        for v in self.views:
            cam = scene.cams[v]
            pr = project(self.params[cam.frame], scene.sh_degree, cam, self.tw, self.th)
            inst, ranges = bin_sort(pr, cam, self.tw, self.th)
            img, T, n, cnt = render(pr, cam, self.tw, self.th, inst, ranges, self.bg)
            self.proj[v], self.inst[v], self.ranges[v] = pr, inst, ranges
            self.image[v], self.T[v], self.n[v], self.counts[v] = img, T, n, cnt

    @property
    def n_gauss(self):
        return self.params.shape[2]

    def visible(self) -> np.ndarray:
        """(F, N) uint8: the set sparse Adam updates -- Gaussians that survive the
        z and det culls in at least one view with a pixel of that view within r
        of the mean on both axes (independent of the tile shape)."""
        F = self.params.shape[0]
        vis = np.zeros((F, self.n_gauss), np.uint8)
        for v in self.views:
            vis[self.scene.cams[v].frame] |= self.proj[v]["visible"].astype(np.uint8)
        return vis

    def loss(self, targets: dict):
        """Mean L1 over all rendered views x pixels x 3 channels and its cotangents."""
        imgs = np.concatenate([self.image[v].reshape(-1) for v in self.views])
        tgts = np.concatenate([np.asarray(targets[v], np.float64).reshape(-1) for v in self.views])
        L, G = loss_l1(imgs, tgts)
        out, o = {}, 0
        for v in self.views:
            k = self.image[v].size
            out[v] = G[o:o + k].reshape(self.image[v].shape)
            o += k
        return L, out

    def backward(self, G: dict, flips: dict | None = None, dynamic="scene"):
        """Texel gradients (F, C, H, W) for cotangents G[v] (3, H, W); also
        returns the per-view 2D gradients."""
        sc = self.scene
        gP = np.zeros_like(self.params)
        g2 = {}
        for v in self.views:
            cam = sc.cams[v]
            g2[v] = backward_view(self.proj[v], cam, self.tw, self.th, self.inst[v], self.ranges[v], G[v],
                                  self.bg, (flips or {}).get(v))
            gpf = np.ascontiguousarray(gP[cam.frame])
            project_backward(self.params[cam.frame], sc.sh_degree, cam, self.proj[v], g2[v], gpf)
            gP[cam.frame] = gpf
        dyn = sc.dynamic if isinstance(dynamic, str) else dynamic
        return scatter(gP, self.ids, dyn, sc.H, sc.W), g2

    def fd(self, G: dict, frame: int, i: int, ch: int, h: float) -> float:
        """Frozen-decision central difference of sum_v <G_v, I_v> in parameter
        ``ch`` of Gaussian ``i`` of ``frame`` (raw texel channel)."""
        sc = self.scene
        tot = 0.0
        for v in self.views:
            cam = sc.cams[v]
            if cam.frame != frame:
                continue
            tot += fd_frozen(self.params[frame], sc.sh_degree, cam, self.tw, self.th, self.proj[v],
                             self.inst[v], self.ranges[v], G[v], i, ch, h, self.bg)
        return tot
