"""Autotuner for the compositing launch shape.

Sweeps tile shape (16x16, 8x32, 32x8; width x height) and Gaussians staged
in LDS per batch (64, 128, 256) on the caller's workload, timing the batched
fwd+bwd chain with HIP events, and keeps the fastest.  Candidates within
`final_margin` of the best first-round time are timed again, with more
repetitions, in two rounds of opposite order, and each keeps its best round:
close shapes are then told apart by more than one short measurement taken
at one moment of the clock's ramp.  Results are cached in a JSON file keyed
by device name and workload (atlas size, Gaussian count, views and their
resolutions), so later runs reuse the choice.
"""
from __future__ import annotations

import hashlib
import json
import os

CANDIDATES = [(16, 16, 64), (16, 16, 128), (16, 16, 256), (8, 32, 64), (8, 32, 128), (8, 32, 256),
              (32, 8, 64), (32, 8, 128), (32, 8, 256)]


def cache_path() -> str:
    return os.environ.get("PACKUV_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "packuv_gs", "tune.json"))


def workload_key(scene, device_name: str) -> str:
    h = hashlib.sha256()
    h.update(f"{scene.W}x{scene.H}x{scene.frames}|{scene.n_gauss}|{scene.sh_degree}".encode())
    for c in scene.cams:
        h.update(f"{c.width}x{c.height}f{c.frame}".encode())
        h.update(bytes(memoryview(c.R.tobytes())))
    return f"{device_name}|{h.hexdigest()[:16]}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def choose(scene, atlas, device="cuda:0", reps=3, candidates=CANDIDATES, use_cache=True,
           final_reps=10, final_margin=0.03):
    """Returns ((tile_w, tile_h, lds_batch), info)."""
    import torch

    from .pipeline import Renderer

    dev = torch.device(device)
    name = torch.cuda.get_device_name(dev)
    key = workload_key(scene, name)
    path = cache_path()
    cache = _load(path) if use_cache else {}
    if key in cache:
        t = tuple(cache[key]["tiling"])
        return t, {"source": "cache", "key": key, "tiling": list(t), "ms": cache[key]["ms"]}
    state = {"target": None, "cap": None}

    def make(cand):
        r = Renderer(scene.occupancy, scene.frames, scene.sh_degree, scene.cams, tiling=cand, batched=True,
                     bg=scene.bg, inst_capacity=state["cap"], device=dev)
        r.forward(atlas)             # grows to the reported count after an overflow
        r.check_overflow = False     # the timed steps below are checked once at the end
        state["cap"] = r.sets[0].cap
        if state["target"] is None:
            state["target"] = torch.rand(3 * r.n_pixels, device=dev, generator=torch.Generator(dev).manual_seed(0))
        r.step(atlas, state["target"])
        torch.cuda.synchronize()
        return r

    def time_steps(r, n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            r.step(atlas, state["target"])
        b.record()
        torch.cuda.synchronize()
        assert r.check(), "instance capacity overflowed while timing"
        return a.elapsed_time(b) / n

    timings = {}
    for cand in candidates:
        r = make(cand)
        timings["x".join(map(str, cand))] = time_steps(r, reps)
        r.close()
        del r
    first = min(timings.values())
    close = [c for c in candidates if timings["x".join(map(str, c))] <= first * (1.0 + final_margin)]
    finalists = sorted(close, key=lambda c: timings["x".join(map(str, c))])[:3]    # at most three held at once
    final = {}
    if len(finalists) > 1:
        rs = [make(c) for c in finalists]
        for order in (range(len(rs)), reversed(range(len(rs)))):
            for k in order:
                ms = time_steps(rs[k], final_reps)
                kk = "x".join(map(str, finalists[k]))
                final[kk] = min(final.get(kk, ms), ms)
        for r in rs:
            r.close()
        del rs
    ranked = final if final else timings
    best = min(ranked, key=ranked.get)
    t = tuple(int(x) for x in best.split("x"))
    if use_cache:
        cache[key] = {"tiling": list(t), "ms": ranked[best], "all_ms": timings, "final_ms": final}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return t, {"source": "sweep", "key": key, "tiling": list(t), "ms": round(ranked[best], 3),
               "all_ms": {k: round(v, 3) for k, v in timings.items()},
               "final_ms": {k: round(v, 3) for k, v in final.items()}}
