"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded scene and compare them.

Comparison rules:
  * discrete outputs (Gaussian ids, culls, tile rectangles, depth keys, sorted
    instance lists, tile ranges) must be bit-identical;
  * projected floats within 1e-6 relative of the FP64 oracle;
  * images and final transmittance within 1e-4 absolute per pixel, except
    pixels "explained" by taking at most two of the oracle's near-threshold
    decisions (relative margin below 1e-4 of q = 9, alpha = 1/255 or
    T = 1e-4) the other way;
  * gradients within 1e-3 relative per element with a floor of 1% of the
    channel's largest magnitude, and 1e-3 relative L2 error per channel, both
    sides using the same cotangent.
"""
from __future__ import annotations

import itertools
import sys

import numpy as np
import torch

import oracle
from paper_2602_23040_amd.pipeline import Renderer

IMG_TOL = 1e-4
BAND = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def renderer(scene, batched=True, tiling=None, cap=None, dynamic="scene", quant_bits=None):
    t = tiling or (scene.tiling.tile_w, scene.tiling.tile_h, scene.tiling.lds_batch)
    dyn = scene.dynamic if dynamic == "scene" else dynamic
    return Renderer(scene.occupancy, scene.frames, scene.sh_degree, scene.cams, tiling=t, batched=batched,
                    bg=scene.bg, dynamic=dyn, inst_capacity=cap, device="cuda:0", quant_bits=quant_bits)


def atlas_tensor(scene):
    return torch.from_numpy(np.ascontiguousarray(scene.atlas, np.float32)).to("cuda:0").reshape(-1)


def run_forward(r, atlas, counters=False):
    r.forward(atlas, counters=counters)
    torch.cuda.synchronize()
    if r.overflowed():
        r.grow_capacity()
        r.forward(atlas, counters=counters)
        torch.cuda.synchronize()
    assert not r.overflowed()


def gpu_images(r):
    img = r.image.cpu().numpy()
    T = r.final_T.cpu().numpy()
    n = r.n_contrib.cpu().numpy()
    out = {}
    for v, c in enumerate(r.cams):
        p0, p1 = r.pix_base[v], r.pix_base[v + 1]
        out[v] = (img[3 * p0:3 * p1].reshape(3, c.height, c.width), T[p0:p1].reshape(c.height, c.width),
                  n[p0:p1].reshape(c.height, c.width))
    return out


def explain(fw, v, gpu_img, gpu_T=None, tol=IMG_TOL, band=BAND, max_pixels=20000):
    """Returns (flips {pixel: positions}, unexplained [(x, y, err)], n_bad).
    A pixel is off when its colour (or, if gpu_T is given, its final
    transmittance) differs from the oracle's by more than tol; it is
    explained when taking at most two of the oracle's near-threshold
    decisions the other way brings every compared value within tol."""
    cam = fw.scene.cams[v]
    err = np.abs(gpu_img - fw.image[v]).max(0)
    if gpu_T is not None:
        err = np.maximum(err, np.abs(gpu_T - fw.T[v]))
    ys, xs = np.nonzero(err > tol)
    flips, unexplained = {}, []
    for x, y in list(zip(xs, ys))[:max_pixels]:
        _, _, _, near = oracle.pixel(fw.proj[v], cam, fw.tw, fw.th, fw.inst[v], fw.ranges[v], x, y, band=band,
                                     bg=fw.bg)
        found = None
        cands = [[k] for k in near] + [list(p) for p in itertools.combinations(near, 2)]
        for fl in cands:
            rgb, T, _, _ = oracle.pixel(fw.proj[v], cam, fw.tw, fw.th, fw.inst[v], fw.ranges[v], x, y, flips=fl,
                                        band=band, bg=fw.bg)
            if np.abs(rgb - gpu_img[:, y, x]).max() <= tol and (gpu_T is None or abs(T - gpu_T[y, x]) <= tol):
                found = fl
                break
        if found is None:
            unexplained.append((int(x), int(y), float(err[y, x])))
        else:
            flips[int(y) * cam.width + int(x)] = found
    return flips, unexplained, int(len(xs))


def grad_compare(g, ref, mask=None, rel=1e-3, floor_frac=0.01):
    """g, ref: (..., C, K) arrays (channel axis -2).  Returns dict of worst stats."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    C = g.shape[-2]
    worst_el, worst_l2, bad = 0.0, 0.0, 0
    bad_channels = {}
    for c in range(C):
        a = g[..., c, :].reshape(-1)
        b = ref[..., c, :].reshape(-1)
        if mask is not None:
            a, b = a[mask.reshape(-1)], b[mask.reshape(-1)]
        mx = np.abs(b).max() if b.size else 0.0
        if mx == 0.0:
            assert np.all(a == 0.0), f"channel {c}: reference is zero but GPU is not"
            continue
        den = np.maximum(np.abs(b), floor_frac * mx)
        r = np.abs(a - b) / den
        worst_el = max(worst_el, float(r.max()))
        nb = int((r > rel).sum())
        bad += nb
        if nb:
            i = int(np.argmax(r))
            bad_channels[c] = (nb, float(r[i]), float(a[i]), float(b[i]), float(mx))
        l2 = np.linalg.norm(a - b) / np.linalg.norm(b)
        worst_l2 = max(worst_l2, float(l2))
    out = {"worst_elem": worst_el, "worst_l2": worst_l2, "n_bad": bad}
    if bad_channels:
        out["bad_channels"] = bad_channels   # channel: (count, worst ratio, got, ref, channel max)
    return out
