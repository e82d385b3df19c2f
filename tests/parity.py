"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded scene and compare them.

Comparison rules:
  * discrete outputs (Gaussian ids, culls, tile rectangles, depth keys, tile
    ranges) must be bit-identical;
  * tile lists: the oracle lists every tile of a rectangle; the GPU drops the
    tiles whose pixel centres all lie outside the ellipse.  Each GPU list must
    be the oracle's list with entries left out and the order kept, and every
    left-out (Gaussian, tile) must have q > 9 at every pixel centre of the
    tile inside the image (FP64 brute force from the oracle's mean and conic);
  * n_contrib is compared after mapping the oracle's list positions onto the
    GPU's lists, exactly on every pixel not explained by a flip; a pixel
    whose count differs (a termination decision at T = 1e-4 can move the
    count while the colour moves by less than 1e-4) must be explained by the
    same flip search, which then has to reproduce the count too;
  * projected floats within 1e-6 relative of the FP64 oracle;
  * images and final transmittance within 1e-4 absolute per pixel, and final
    transmittance within 2e-3 relative (a decision taken the other way at a
    deep pixel moves T by at least 1/255 of itself while its colour may move
    by less than 1e-4), except pixels "explained" by taking at most two of the
    oracle's near-threshold decisions (relative margin below 1e-4 of q = 9,
    alpha = 1/255 or T = 1e-4) the other way;
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
# Relative tolerance on final transmittance.  A compositing decision taken the
# other way multiplies T by 1 - alpha with alpha >= 1/255, a relative change of
# at least 3.9e-3; FP32 rounding of the product stays below about 5e-4 even
# where alphas near the 0.99 clamp amplify it (1 - alpha has 1 / (1 - alpha)
# times alpha's relative error).
T_REL = 2e-3


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
    """Eager forward; an overflow grows the buffers and renders again inside
    Renderer.forward, so the step must end without one."""
    r.forward(atlas, counters=counters)
    torch.cuda.synchronize()
    assert r.check()


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


def _n_map(fw, v, kept):
    """Maps the oracle's n_contrib at pixel (x, y) (a position in the
    oracle's tile list) to a position in the GPU's list, which is the
    oracle's with the kept flags applied (identity for kept = None)."""
    if kept is None:
        return lambda x, y, n: n
    cam = fw.scene.cams[v]
    TX = (cam.width + fw.tw - 1) // fw.tw
    ck = np.concatenate([[0], np.cumsum(kept, dtype=np.int64)])

    def f(x, y, n):
        if n <= 0:
            return 0
        s = int(fw.ranges[v][(y // fw.th) * TX + x // fw.tw, 0])
        return int(ck[s + n] - ck[s])
    return f


def explain(fw, v, gpu_img, gpu_T=None, gpu_n=None, kept=None, tol=IMG_TOL, band=BAND, max_pixels=20000):
    """Returns (flips {pixel: positions}, unexplained [(x, y, err)], n_bad).
    A pixel is off when its colour differs from the oracle's by more than tol,
    or, if gpu_T is given, its final transmittance by more than tol or by
    more than T_REL relative, or, if gpu_n
    is given, when its n_contrib differs from the oracle's moved onto the
    GPU's lists (kept flags from check_tile_lists).  It is explained when
    taking at most two of the oracle's near-threshold decisions the other
    way brings every compared value within tol and, with gpu_n, makes the
    count equal.  More than max_pixels off pixels in one view is a failure,
    not a sample."""
    cam = fw.scene.cams[v]
    err = np.abs(gpu_img - fw.image[v]).max(0)
    off = err > tol
    if gpu_T is not None:
        dT = np.abs(gpu_T - fw.T[v])
        err = np.maximum(err, dT)
        # a decision taken the other way scales T by (1 - alpha), alpha >= 1/255, a
        # relative change far above FP32 rounding: deep pixels (small T) show it in T
        # even when the colour moves by less than tol
        off |= (dT > tol) | (dT > T_REL * fw.T[v])
    if gpu_n is not None:
        exp_n = gpu_n_contrib(fw, v, kept) if kept is not None else fw.n[v]
        off |= gpu_n != exp_n
    nmap = _n_map(fw, v, kept)
    ys, xs = np.nonzero(off)
    assert len(xs) <= max_pixels, f"view {v}: {len(xs)} pixels off (more than {max_pixels} to examine)"
    flips, unexplained = {}, []
    for x, y in zip(xs, ys):
        _, _, _, near = oracle.pixel(fw.proj[v], cam, fw.tw, fw.th, fw.inst[v], fw.ranges[v], x, y, band=band,
                                     bg=fw.bg)
        found = None
        cands = [[k] for k in near] + [list(p) for p in itertools.combinations(near, 2)]
        for fl in cands:
            rgb, T, n, _ = oracle.pixel(fw.proj[v], cam, fw.tw, fw.th, fw.inst[v], fw.ranges[v], x, y, flips=fl,
                                        band=band, bg=fw.bg)
            if np.abs(rgb - gpu_img[:, y, x]).max() > tol:
                continue
            if gpu_T is not None and abs(T - gpu_T[y, x]) > min(tol, T_REL * T):
                continue
            if gpu_n is not None and nmap(int(x), int(y), n) != int(gpu_n[y, x]):
                continue
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


def _q_outside_footprint(pr, cam, tw, th, tiles, ids, chunk=4096):
    """Least FP64 q over the in-image pixel centres of tile tiles[k] for
    Gaussian ids[k], minimised over k (inf for no pairs)."""
    TX = (cam.width + tw - 1) // tw
    lx, ly = np.arange(tw) + 0.5, np.arange(th) + 0.5
    qmin = np.inf
    for s0 in range(0, len(tiles), chunk):
        t = np.asarray(tiles[s0:s0 + chunk], np.int64)
        i = np.asarray(ids[s0:s0 + chunk], np.int64)
        X = ((t % TX) * tw)[:, None] + lx[None, :]
        Y = ((t // TX) * th)[:, None] + ly[None, :]
        dx = (X - pr["mean"][i, 0][:, None])[:, None, :]
        dy = (Y - pr["mean"][i, 1][:, None])[:, :, None]
        a, b, c = (pr["conic"][i, k][:, None, None] for k in range(3))
        q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
        inside = (X < cam.width)[:, None, :] & (Y < cam.height)[:, :, None]
        q = np.where(inside, q, np.inf)
        qmin = min(qmin, float(q.min()))
    return qmin


def check_tile_lists(fw, v, keys, vals, tile_base, N):
    """View v's sorted GPU instances (keys: global tile ids ascending, vals:
    v N + Gaussian id) against the oracle's tile lists, which hold every tile
    of each rectangle.  Asserts that each GPU list is the oracle's with some
    entries left out and the order kept, and that every left-out
    (Gaussian, tile) has q > 9 at every pixel centre of the tile inside the
    image.  Returns the oracle instances' kept flags."""
    cam, inst = fw.scene.cams[v], fw.inst[v]
    lo = int(np.searchsorted(keys, np.uint32(tile_base[v]), "left"))
    hi = int(np.searchsorted(keys, np.uint32(tile_base[v + 1]), "left"))
    gt = keys[lo:hi].astype(np.int64) - int(tile_base[v])
    gi = vals[lo:hi].astype(np.int64) - v * N
    assert gi.size == 0 or (gi.min() >= 0 and gi.max() < N), f"view {v}: GPU values outside the view's records"
    ocode = (inst["tile"].astype(np.int64) << 28) | inst["id"].astype(np.int64)
    gcode = (gt << 28) | gi
    kept = np.isin(ocode, gcode)
    assert np.array_equal(ocode[kept], gcode), f"view {v}: GPU tile lists are not order-kept sublists of the oracle's"
    dropped = np.flatnonzero(~kept)
    qmin = _q_outside_footprint(fw.proj[v], cam, fw.tw, fw.th, inst["tile"][dropped], inst["id"][dropped])
    assert qmin > 9.0, f"view {v}: a dropped tile has a pixel centre with q = {qmin} <= 9"
    say(f"[lists] view {v}: {len(inst)} oracle instances, {int(kept.sum())} kept by the GPU, "
        f"{len(dropped)} dropped (least q over dropped tiles {qmin:.4f})")
    return kept


def gpu_n_contrib(fw, v, kept):
    """The oracle's n_contrib of view v (list positions reached: where the
    pixel stopped, else its tile list's length) moved to positions in the
    GPU's lists, which are the oracle's with the kept flags applied: the
    number of kept entries before that position (the Gaussian a pixel stops
    at has q <= 9 there, so its tile is kept for it)."""
    cam = fw.scene.cams[v]
    TX = (cam.width + fw.tw - 1) // fw.tw
    ck = np.concatenate([[0], np.cumsum(kept, dtype=np.int64)])
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    start = fw.ranges[v][(ys // fw.th) * TX + xs // fw.tw, 0]
    n = fw.n[v].astype(np.int64)
    return ck[start + n] - ck[start]


def check_records(fw, v, bins, tsets, splats, N):
    """View v's projection records against the oracle: every record the GPU
    lists is one the oracle lists, with the same rectangle and depth key; its
    kept tiles lie in the rectangle (a mask of the rectangle's bits, or every
    tile for rectangles of more than 64 tiles); culled records are zero; FP64
    means are equal wherever the oracle projects the Gaussian."""
    pr = fw.proj[v]
    sl = slice(v * N, (v + 1) * N)
    b, ts, s = bins[sl], tsets[sl], splats[sl]
    valid = pr["valid"] == 1
    listed = b["n_tiles"] > 0
    assert np.all(valid[listed]), f"view {v}: the GPU lists a record the oracle culls"
    assert np.array_equal(b["rect"][listed], pr["rect"][listed].astype(np.int16))
    assert np.array_equal(b["key"][listed], pr["key"][listed])
    w = pr["rect"][:, 2] - pr["rect"][:, 0] + 1
    h = pr["rect"][:, 3] - pr["rect"][:, 1] + 1
    area = (w * h).astype(np.int64)
    assert np.array_equal(area[valid], pr["n_tiles"][valid])
    assert np.all(b["n_tiles"][listed] <= area[listed])
    small = listed & (area <= 64)
    mask = ts["mask"]
    assert np.array_equal(np.bitwise_count(mask[small]).astype(np.int64), b["n_tiles"][small].astype(np.int64))
    assert np.all((mask[small] >> area[small].astype(np.uint64)) == 0), f"view {v}: kept tiles outside the rectangle"
    big = listed & (area > 64)
    assert np.all(mask[big] == 0) and np.array_equal(b["n_tiles"][big], area[big])
    assert np.array_equal(ts["x_lo"][listed], pr["rect"][listed, 0]) and np.array_equal(ts["y_lo"][listed], pr["rect"][listed, 1])
    assert np.array_equal(ts["width"][listed], w[listed]) and np.array_equal(ts["height"][listed], h[listed])
    assert not ts.view(np.uint8).reshape(-1, 16)[~listed].any(), f"view {v}: culled tile sets not zero"
    assert not b.view(np.uint8).reshape(-1, 16)[~listed].any(), f"view {v}: culled bins not zero"
    assert np.array_equal(s["mean"][valid], pr["mean"][valid]), f"view {v}: FP64 means differ"
    return valid, listed
