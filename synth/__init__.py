"""Seeded synthetic scenes for the PackUV-GS splatting path.

This module only draws inputs: UV-atlas texels, occupancy and dynamic masks,
and pinhole cameras.  It holds none of the method's arithmetic (no activation,
projection, binning or compositing), so that both the CPU oracle and the GPU
library can consume the very same arrays.

Texel channel order (one atlas per frame, planar ``[F][C][H][W]`` float32):

====  =========================================================
 0-2  position x, y, z (world units)
 3-5  log-scales l_sx, l_sy, l_sz
 6-9  rotation quaternion (w, x, y, z), real part first
  10  logit-opacity
 11+  SH coefficients k[j][ch], j = 0..(L+1)^2-1, ch = R, G, B
      (channel 11 + 3*j + ch)
====  =========================================================

The record is the 3DGS primitive of the paper's preliminaries (position,
covariance from scale and rotation, opacity, SH colour), stored per texel as
in the "Fitting UV Maps Directly" paragraph (Sec. 4.2), with the Cartesian
position the low-precision-optimisation paragraph quantises (Sec. 4.3).

Cameras are OpenCV pinholes: ``x_c = R x + t`` with x right, y down, z
forward; a horizontal field of view of 60 degrees gives
``fx = fy = W / (2 tan 30deg)``, ``cx = W/2``, ``cy = H/2``.

The five workloads mirror the multi-camera captures the paper fits (50+
camera 360-degree rigs, 1920x1200 frames downsampled to ~1.6K, 1024^2 UV maps,
300K-500K Gaussians per frame); they stand in for the datasets, which are not
reproduced here.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

N_BASE_CHANNELS = 11


def n_channels(sh_degree: int) -> int:
    return N_BASE_CHANNELS + 3 * (sh_degree + 1) ** 2


@dataclass
class Camera:
    R: np.ndarray          # (3, 3) float64, world -> camera rotation (rows = camera axes)
    t: np.ndarray          # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    frame: int = 0


@dataclass
class Tiling:
    tile_w: int = 16
    tile_h: int = 16
    lds_batch: int = 256


@dataclass
class Scene:
    name: str
    atlas: np.ndarray               # (F, C, H, W) float32, 0 on unoccupied texels
    occupancy: np.ndarray           # (H, W) uint8, shared by every frame of the window
    cams: list                      # list[Camera]
    sh_degree: int
    tiling: Tiling = field(default_factory=Tiling)
    dynamic: np.ndarray | None = None   # (H, W) uint8 gradient-freeze mask, or None (all dynamic)
    bg: tuple = (0.0, 0.0, 0.0)
    seed: int = 0

    @property
    def frames(self) -> int:
        return self.atlas.shape[0]

    @property
    def C(self) -> int:
        return self.atlas.shape[1]

    @property
    def H(self) -> int:
        return self.atlas.shape[2]

    @property
    def W(self) -> int:
        return self.atlas.shape[3]

    @property
    def n_gauss(self) -> int:
        return int(np.count_nonzero(self.occupancy))

    @property
    def n_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cams))

    def sha256(self) -> dict:
        out = {"atlas": hashlib.sha256(self.atlas.tobytes()).hexdigest(),
               "occupancy": hashlib.sha256(self.occupancy.tobytes()).hexdigest()}
        if self.dynamic is not None:
            out["dynamic"] = hashlib.sha256(self.dynamic.tobytes()).hexdigest()
        return out


# ----------------------------------------------------------------------------- cameras

def focal_for_hfov(width: int, hfov_deg: float = 60.0) -> float:
    return width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))


def pinhole(R, t, width, height, frame=0, hfov_deg=60.0) -> Camera:
    f = focal_for_hfov(width, hfov_deg)
    return Camera(R=np.asarray(R, np.float64).reshape(3, 3).copy(),
                  t=np.asarray(t, np.float64).reshape(3).copy(),
                  fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height), frame=int(frame))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for an OpenCV camera at ``eye`` looking at ``target``."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return R, t


def ring_cameras(n, radius, width, height, frame=0, sizes=None):
    cams = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        R, t = look_at(radius * np.array([math.cos(a), math.sin(a), 0.0]))
        w, h = sizes[k % len(sizes)] if sizes else (width, height)
        cams.append(pinhole(R, t, w, h, frame))
    return cams


def fibonacci_cameras(n, radius, width, height, frame=0):
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for k in range(n):
        z = 1.0 - 2.0 * (k + 0.5) / n
        rho = math.sqrt(max(0.0, 1.0 - z * z))
        phi = k * golden
        eye = radius * np.array([rho * math.cos(phi), rho * math.sin(phi), z])
        R, t = look_at(eye)
        cams.append(pinhole(R, t, width, height, frame))
    return cams


# ----------------------------------------------------------------------------- texels

def _unit_quaternions(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def fill_texels(rng, occupancy, sh_degree, pos_lo, pos_hi, lscale_mu, lscale_sd,
                lopac_mu=0.0, lopac_sd=1.0, sh_sd=0.2, rgb_dc=False):
    """Draw one frame of texels.  Draw order: position, log-scale, quaternion,
    logit-opacity, SH.  Only occupied texels (row-major order) get values."""
    H, W = occupancy.shape
    C = n_channels(sh_degree)
    idx = np.flatnonzero(occupancy.reshape(-1))
    n = idx.size
    vals = np.zeros((C, n), np.float64)
    vals[0:3] = rng.uniform(np.asarray(pos_lo)[:, None], np.asarray(pos_hi)[:, None], (3, n))
    vals[3:6] = rng.normal(lscale_mu, lscale_sd, (3, n))
    vals[6:10] = _unit_quaternions(rng, n).T
    vals[10] = rng.normal(lopac_mu, lopac_sd, n)
    nsh = 3 * (sh_degree + 1) ** 2
    if rgb_dc:
        # "SH degree-0 RGB U(0,1)": the base colour the Gaussian shows, stored as the
        # DC coefficient that yields it (colour = 0.5 + Y_00 k, Y_00 = 1/(2 sqrt(pi))).
        rgb = rng.uniform(0.0, 1.0, (3, n))
        vals[11:11 + 3] = (rgb - 0.5) * (2.0 * math.sqrt(math.pi))
        if nsh > 3:
            vals[14:11 + nsh] = rng.normal(0.0, sh_sd, (nsh - 3, n))
    else:
        vals[11:11 + nsh] = rng.normal(0.0, sh_sd, (nsh, n))
    atlas = np.zeros((C, H * W), np.float32)
    atlas[:, idx] = vals.astype(np.float32)
    return atlas.reshape(C, H, W)


# ----------------------------------------------------------------------------- configs

CONFIG_NAMES = {
    1: "plain-1view-64sq-atlas-128sq",
    2: "ring8-256sq-atlas-sh3-512sq",
    3: "fib50-multiscale-344k-slots-1024x768",
    4: "temporal-16f-x-8ring-1024sq-atlas-1080p-720p",
    5: "fib50-2048sq-atlas-1080p-adam",
}


def multiscale_slots(levels=((512, 512), (256, 256), (128, 128))):
    """Slot mask of a horizontal-strip atlas: level 0 on the right, the finer
    levels left of it, top-aligned (atlas width = sum of level widths, height =
    max level height)."""
    (h0, w0), rest = levels[0], levels[1:]
    W = w0 + sum(w for _, w in rest)
    H = max(h for h, _ in levels)
    slots = np.zeros((H, W), np.uint8)
    x = 0
    for h, w in rest:
        slots[:h, x:x + w] = 1
        x += w
    slots[:h0, x:x + w0] = 1
    return slots


def make_scene(config: int, seed: int | None = None, target: bool = False) -> Scene:
    """Scene for one of the five workloads.  ``target=True`` draws the second
    seeded Gaussian set (seed + 500) used to render the L1 target."""
    if seed is None:
        seed = config
    if target:
        seed += 500
    rng = np.random.default_rng(seed)
    if config == 1:
        occ = np.ones((64, 64), np.uint8)
        atlas = fill_texels(rng, occ, 0, (-1, -1, 2), (1, 1, 4), -4.0, 0.5, rgb_dc=True)
        cams = [pinhole(np.eye(3), np.zeros(3), 128, 128)]
        return Scene(CONFIG_NAMES[1], atlas[None], occ, cams, 0, Tiling(16, 16, 256), seed=seed)
    if config == 2:
        occ = np.ones((256, 256), np.uint8)
        atlas = fill_texels(rng, occ, 3, (-1, -1, -1), (1, 1, 1), -5.0, 0.5)
        cams = ring_cameras(8, 4.0, 512, 512)
        return Scene(CONFIG_NAMES[2], atlas[None], occ, cams, 3, Tiling(16, 16, 256), seed=seed)
    if config == 3:
        mrng = np.random.default_rng(200 + config)
        slots = multiscale_slots()
        occ = (slots & (mrng.random(slots.shape) < 0.85)).astype(np.uint8)
        atlas = fill_texels(rng, occ, 3, (-1, -1, -1), (1, 1, 1), -5.0, 0.5)
        cams = fibonacci_cameras(50, 4.0, 1024, 768)
        return Scene(CONFIG_NAMES[3], atlas[None], occ, cams, 3, Tiling(16, 16, 256), seed=seed)
    if config == 4:
        return _temporal_scene(seed, rng)
    if config == 5:
        mrng = np.random.default_rng(200 + config)
        occ = (mrng.random((2048, 2048)) < 0.75).astype(np.uint8)
        atlas = fill_texels(rng, occ, 3, (-1, -1, -1), (1, 1, 1), -6.0, 0.7, lopac_mu=1.0)
        cams = fibonacci_cameras(50, 4.0, 1920, 1080)
        return Scene(CONFIG_NAMES[5], atlas[None], occ, cams, 3, Tiling(16, 16, 256), seed=seed)
    raise ValueError(f"unknown config {config}")


def _temporal_scene(seed, rng, frames=16, side=1024, views_per_frame=8):
    mrng = np.random.default_rng(200 + 4)
    occ = (mrng.random((side, side)) < 0.60).astype(np.uint8)
    base = fill_texels(rng, occ, 3, (-1, -1, -1), (1, 1, 1), -5.0, 0.5)
    idx = np.flatnonzero(occ.reshape(-1))
    mu = base.reshape(base.shape[0], -1)[0:3, idx].astype(np.float64)      # (3, n)
    frng = np.random.default_rng(300 + 4)
    centre = frng.uniform(-0.5, 0.5, 3)
    d2 = ((mu - centre[:, None]) ** 2).sum(0)
    n_dyn = int(round(0.2 * idx.size))
    dyn_sel = np.argsort(d2, kind="stable")[:n_dyn]
    dynamic = np.zeros(side * side, np.uint8)
    dynamic[idx[dyn_sel]] = 1
    # smooth flow: (0.05/8) * sum_j v_j sin(2 pi kappa_j . mu + omega_j f + phi_j)
    v = frng.standard_normal((8, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    kap = frng.normal(0.0, 0.25, (8, 3))
    omega = frng.uniform(0.1, 0.5, 8)
    phase = frng.uniform(0.0, 2.0 * math.pi, 8)
    mu_d = mu[:, dyn_sel]
    atlas = np.repeat(base[None], frames, axis=0)
    for f in range(frames):
        arg = 2.0 * math.pi * (kap @ mu_d) + (omega * f + phase)[:, None]       # (8, n_dyn)
        disp = (0.05 / 8.0) * (v.T @ np.sin(arg))                               # (3, n_dyn)
        plane = atlas[f].reshape(atlas.shape[1], -1)
        plane[0:3, idx[dyn_sel]] = (mu_d + disp).astype(np.float32)
    cams = []
    for f in range(frames):
        cams += ring_cameras(views_per_frame, 4.0, 0, 0, frame=f,
                             sizes=[(1920, 1080), (1280, 720)])
    return Scene(CONFIG_NAMES[4], atlas, occ, cams, 3, Tiling(16, 16, 256),
                 dynamic=dynamic.reshape(side, side), seed=seed)


def random_scene(side=16, sh_degree=0, views=1, width=64, height=48, seed=0,
                 occupancy=1.0, lscale=(-3.0, 0.4), pos=((-1, -1, -1), (1, 1, 1)),
                 radius=4.0, lopac=(0.0, 1.0), frames=1, tiling=None, dynamic_frac=None):
    """Small scene for tests: ``side``^2 atlas, ring cameras (or identity camera
    when ``views == 0`` is replaced by one camera at the origin looking down +z)."""
    rng = np.random.default_rng(seed)
    mrng = np.random.default_rng(seed + 1000)
    occ = (mrng.random((side, side)) < occupancy).astype(np.uint8) if occupancy < 1.0 \
        else np.ones((side, side), np.uint8)
    planes = []
    for _ in range(frames):
        planes.append(fill_texels(rng, occ, sh_degree, pos[0], pos[1], lscale[0], lscale[1],
                                  lopac_mu=lopac[0], lopac_sd=lopac[1]))
    atlas = np.stack(planes)
    cams = []
    for f in range(frames):
        if views == 0:
            cams.append(pinhole(np.eye(3), np.zeros(3), width, height, frame=f))
        else:
            cams += ring_cameras(views, radius, width, height, frame=f)
    dyn = None
    if dynamic_frac is not None:
        dyn = ((mrng.random((side, side)) < dynamic_frac) & (occ > 0)).astype(np.uint8)
    return Scene(f"random-{side}-{seed}", atlas, occ, cams, sh_degree,
                 tiling or Tiling(16, 16, 64), dynamic=dyn, seed=seed)


def flow_masks(scene: Scene, seed: int, coverage: float = 0.2, mean_radius: float = 0.06) -> np.ndarray:
    """Seeded stand-ins for per-camera motion masks (the thresholded, dilated
    optical flow the paper computes from video, which this workload does not
    have): for every view, random discs until about `coverage` of its pixels
    are set.  Returns uint8 [n_pixels], the views' [H][W] masks concatenated in
    view order (the layout of the rendered per-pixel buffers)."""
    rng = np.random.default_rng(seed)
    out = []
    for cam in scene.cams:
        H, W = cam.height, cam.width
        m = np.zeros((H, W), np.uint8)
        set_px, target = 0, coverage * H * W
        while set_px < target:
            cx, cy = rng.uniform(0, W), rng.uniform(0, H)
            r = rng.uniform(0.5, 1.5) * mean_radius * min(H, W)
            x0, x1 = max(0, int(cx - r)), min(W, int(cx + r) + 1)
            y0, y1 = max(0, int(cy - r)), min(H, int(cy + r) + 1)
            yy, xx = np.ogrid[y0:y1, x0:x1]
            sub = m[y0:y1, x0:x1]
            disc = (xx + 0.0 - cx) ** 2 + (yy + 0.0 - cy) ** 2 <= r * r
            set_px += int(np.count_nonzero(disc & (sub == 0)))
            sub[disc] = 1
        out.append(m.reshape(-1))
    return np.concatenate(out) if out else np.zeros(0, np.uint8)
