"""Benchmark: fwd+bwd throughput of PackUV-GS splatting on one MI355X.

Workload (default): 50 views at 1024x768 on a Fibonacci sphere (radius 4)
around a three-level multi-scale atlas (512^2 + 256^2 + 128^2 slots in an
896x512 strip, 85% occupied -> 292,614 Gaussians, SH degree 3), i.e. the
batched-vs-plain configuration.  One step = atlas fetch, projection, tile
bin + depth sort, compositing, L1 loss against a target rendered from a
second seeded Gaussian set, and the adjoint back to the atlas.

* batched: every view in one call chain, captured once in a HIP graph and
  replayed (no host synchronisation inside a step);
* plain: the same kernels one view at a time, one instance-count
  synchronisation per view, no graph.

Prints one JSON line (rank 0).  ``value`` is the batched rate in Mpixels/s
(pixels rendered forward and backward per second); Gaussian-view
projections per second, the plain rate and the speedup are reported beside
it.  ``roofline`` describes the kernel that takes the most time per step,
timed live with HIP events on the stream it is launched on; ``cpu_baseline``
is the FP64 CPU oracle timed on a bounded sample of views, whose images also
serve as a parity spot check of the GPU run.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# FP32 operations per evaluated (pixel, Gaussian) pair and per composited pair in
# the compositing loop: dx, dy (2) + quadratic form (a dx: 1, fma: 2, c dy dy: 2,
# fma: 2) = 9; composited: -q/2, exp, o e, 1 - alpha, T (1 - alpha), T alpha,
# three colour FMAs (6) = 12.
FLOP_EVAL = 9
FLOP_COMP = 12
# FP32 operations per composited pair in the compositing adjoint: dx, dy (2),
# q (7), alpha (-q/2, exp, o e, clamp: 4), 1 - alpha, its reciprocal, T_k (3),
# T alpha (1), colour moments (3 FMA: 6), G . c - S (3 FMA: 6), S update
# (FMA: 2), dq' = alpha dL/dalpha = T alpha (G . c - S) (1), opacity moment
# sum dq' (1), dq' (dx, dy) (2), first moments (2), second moments (3 FMA: 6)
# = 43.  (S = G . B is the colour behind the Gaussian projected on the pixel's
# colour cotangent G; dL/do = sum dq' / o is formed per record.)
FLOP_BWD = 43
# Bytes per radix pass and instance: upsweep reads the key (8), downsweep reads
# key + value (12) and writes them (12).
SORT_BYTES_PER_PASS = 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3, help="0 skips the plain (per-view) leg")
    ap.add_argument("--tiling", type=str, default="auto", help="auto (autotuner) or WxHxB, e.g. 16x16x256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-lpo", action="store_true",
                    help="skip the step with the LPO fake quantiser and the flow-masking timing (reported under "
                         "'lpo' and 'flow_mask')")
    ap.add_argument("--also-configs", type=str, default="",
                    help="comma-separated workload numbers (2, 4, 5) whose batched and plain steps are also timed "
                         "and reported under 'other_configs' (off by default: config 4 and 5 scenes take a minute "
                         "to build)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (a reference of known "
                         "size for the HBM traffic counters) and exit")
    return ap.parse_args()


def recorded_traffic(kernel, workload, tiling):
    """HBM bytes per launch of `kernel` from the committed counter record
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE of the same launch,
    scaled by what the counters read for a copy of known size), or None when
    there is no record for this workload and tiling or the kernel's source or
    its build flags (the build script) have changed since the counters were
    taken."""
    import hashlib

    def digest(path):
        with open(os.path.join(ROOT, path), "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()

    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f)[f"{kernel}|{workload}|{tiling}"]
        same = digest(rec["source"]) == rec["source_sha256"] and digest(rec["build"]) == rec["build_sha256"]
    except (OSError, KeyError, ValueError):
        return None
    return rec["bytes_per_launch"] if same else None


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n * 4, "reads_per_copy": n * 4, "writes_per_copy": n * 4}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; sharding the views over several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2602_23040_amd import autotune
    from paper_2602_23040_amd.pipeline import Renderer

    dev = torch.device("cuda:0")
    sc = synth.make_scene(args.config)
    tgt_sc = synth.make_scene(args.config, target=True)
    V = len(sc.cams)
    N = sc.n_gauss
    atlas = torch.from_numpy(np.ascontiguousarray(sc.atlas).reshape(-1)).to(dev)
    tgt_atlas = torch.from_numpy(np.ascontiguousarray(tgt_sc.atlas).reshape(-1)).to(dev)

    # --- tiling: autotuner (cached) or fixed
    if args.tiling == "auto":
        tiling, tune_info = autotune.choose(sc, atlas, device=dev)
    else:
        tiling = tuple(int(x) for x in args.tiling.split("x"))
        tune_info = {"source": "fixed"}

    def make(batched, cap=None):
        r = Renderer(sc.occupancy, sc.frames, sc.sh_degree, sc.cams, tiling=tiling, batched=batched, bg=sc.bg,
                     dynamic=sc.dynamic, inst_capacity=cap, device=dev)
        r.forward(atlas)             # an overflow here grows the buffers to the reported count and renders again
        r.check_overflow = False     # timed eager steps: checked once after the timed region
        return r

    # target image: the second seeded Gaussian set rendered by the same path (setup, untimed)
    rt = Renderer(tgt_sc.occupancy, tgt_sc.frames, tgt_sc.sh_degree, tgt_sc.cams, tiling=tiling, device=dev)
    rt.forward(tgt_atlas)
    torch.cuda.synchronize()
    target = rt.image.clone()
    rt.close()
    del rt

    rb = make(True)
    # counts for the algorithmic work of one step (one untimed pass with counters)
    rb.forward(atlas, counters=True)
    torch.cuda.synchronize()
    n_eval, n_comp = (int(x) for x in rb.counters.cpu().tolist())
    n_inst = int(rb.sets[0].n_inst[0].item())
    s0 = rb.sets[0]
    n_rec = int((s0.bins[:4 * s0.info.n_gv].view(-1, 4)[:, 3] > 0).sum().item())   # records keeping a tile
    P = rb.n_pixels

    stream = torch.cuda.current_stream()
    if args.no_graph:
        def run_step():
            rb.step(atlas, target)
    else:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            rb.step(atlas, target)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            rb.step(atlas, target)
        torch.cuda.synchronize()

        def run_step():
            graph.replay()

    for _ in range(args.warmup):
        run_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run_step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    assert rb.check(), "instance capacity overflowed inside the timed region"
    # spread of single steps (after the timed region): each step between its own events
    dist = step_spread(run_step, max(10, args.steps))
    loss = float(rb.loss.item())

    # --- per-kernel live timing of the step's stages (same stream, eager calls)
    stages = stage_times(rb, atlas, target, reps=5)

    # --- plain path: same kernels one view at a time (--plain-steps 0 skips it)
    ms_plain = ms_plain_graph = None
    same_img = None
    if args.plain_steps > 0:
        rp = make(False)
        rp.step(atlas, target)
        torch.cuda.synchronize()
        t0p = time.perf_counter()
        for _ in range(args.plain_steps):
            rp.step(atlas, target)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0p) * 1e3 / args.plain_steps
        same_img = bool(torch.equal(rp.image, rb.image))
        # plain + graph: the same per-view chain captured once its capacities are known
        if not args.no_graph:
            rp.plain_sync = False
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                rp.step(atlas, target)
            stream.wait_stream(side)
            torch.cuda.synchronize()
            pg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(pg):
                rp.step(atlas, target)
            pg.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.plain_steps):
                pg.replay()
            e1.record()
            torch.cuda.synchronize()
            assert rp.check(), "plain capacities overflowed under graph replay"
            ms_plain_graph = e0.elapsed_time(e1) / args.plain_steps
            del pg
        rp.close()

    # --- roofline for the stage with the largest time share
    sort_passes = rb.sets[0].info.sort_passes
    work = {
        "render_fwd": ("alu", (FLOP_EVAL * n_eval + FLOP_COMP * n_comp) / 1e12, "TFLOP/s", PEAK_FP32_TFLOPS),
        "render_bwd": ("alu", FLOP_BWD * n_comp / 1e12, "TFLOP/s", PEAK_FP32_TFLOPS),
        "bin_sort": ("hbm", (SORT_BYTES_PER_PASS * sort_passes * n_inst + 28 * n_inst) / 1e9, "GB/s", PEAK_HBM_GBS),
        "project": ("hbm", (4 * sc.C * N + 80 * N * V) / 1e9, "GB/s", PEAK_HBM_GBS),
    }
    dom = max(stages, key=lambda k: stages[k])
    roof = None
    if dom in work:
        bound, amount, unit, peak = work[dom]
        achieved = amount / (stages[dom] / 1e3)
        roof = {"kernel": dom, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4),
                "traffic": recorded_traffic(dom, sc.name, "x".join(str(x) for x in tiling)),
                "ms": round(stages[dom], 4)}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": None, "traffic": None, "ms": round(stages[dom], 4)}

    cpu = None if args.no_cpu_baseline else cpu_baseline(sc, rb, target, args.cpu_seconds)
    lpo = None if args.no_lpo else lpo_leg(sc, atlas, target, tiling, args.steps, args.warmup, not args.no_graph)
    fmask = None if args.no_lpo else flow_mask_leg(sc, rb, atlas)
    uvp = None if args.no_lpo else uv_prune_leg(sc, rb, atlas)
    objective = None if args.no_lpo else objective_leg(sc, rb, atlas, target, tiling, args.steps, args.warmup,
                                                       not args.no_graph)

    out = {
        "metric": "fwd+bwd Mpixels/s & Gaussians/s, batched vs plain, at oracle-matched tolerance",
        "value": round(P / ms / 1e3, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "atlas": f"{sc.W}x{sc.H}", "gaussians": N, "views": V,
                   "resolution": f"{sc.cams[0].width}x{sc.cams[0].height}", "sh_degree": sc.sh_degree,
                   "tiling": "x".join(str(t) for t in tiling), "graph": not args.no_graph},
        "gaussians_per_s": round(N * V / ms * 1e3, 1),
        "plain": None if ms_plain is None else {
            "ms_per_step": round(ms_plain, 3), "mpixels_per_s": round(P / ms_plain / 1e3, 2),
            "gaussians_per_s": round(N * V / ms_plain * 1e3, 1), "image_bitwise_equal": same_img,
            "graph_ms_per_step": None if ms_plain_graph is None else round(ms_plain_graph, 3)},
        "step_ms_spread": dist,
        "speedup_vs_plain": None if ms_plain is None else round(ms_plain / ms, 3),
        "wall_s_timed": round(wall, 4),
        "work": {"instances": n_inst, "records": n_rec, "pairs_evaluated": n_eval, "pairs_composited": n_comp, "pixels": P,
                 "loss": loss},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "lpo": lpo,
        "flow_mask": fmask,
        "full_objective": objective,
        "uv_prune": uvp,
        "autotune": tune_info,
    }
    rb.close()
    if args.also_configs:
        rp = rb = None
        torch.cuda.empty_cache()
        out["other_configs"] = [other_config(int(c), None if args.tiling == "auto" else tiling, max(2, args.steps // 4), 2)
                                for c in args.also_configs.split(",") if c.strip()]
    print(json.dumps(out), flush=True)


# Algorithmic FP32 operations per pixel and channel of the photometric loss:
# five separable window sums (2 passes x 11 taps x 2 flop each), the SSIM
# value and its three partials (~40), and the separable adjoint blur of the
# three partial maps (3 x 2 x 11 x 2).  The kernel recomputes the halo of
# each 32 x 32 block (about 1.6 times this), which is not counted.
FLOP_PHOTO = 5 * 2 * 11 * 2 + 40 + 3 * 2 * 11 * 2
LAMBDA_SSIM = 0.2      # 3DGS's weight (the paper does not give one)
S_MAX = 0.05           # scale cap for the scale regulariser (not given either)


def step_spread(run_step, reps):
    """Median, p10 and p90 of `reps` single steps, each between its own events."""
    import numpy as np
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        run_step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)])
    return {"reps": reps, "median": round(float(np.median(t)), 4), "p10": round(float(np.percentile(t, 10)), 4),
            "p90": round(float(np.percentile(t, 90)), 4)}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def uv_prune_leg(sc, r, atlas, M=512, Nv=256, K=2, reps=5):
    """UV-based pruning of the workload's Gaussians on an M x Nv map (top K by
    opacity per pixel), timed with events; HBM-bound: two stable radix sorts
    of (key, index) pairs over the Gaussians plus a gather of their position
    and opacity."""
    import torch
    from paper_2602_23040_amd import _abi as abi
    stream = torch.cuda.current_stream()
    uv, rank, keep = r.uv_prune(atlas, M, Nv, K)
    torch.cuda.synchronize()
    kept = int(keep.sum().item())
    n = r.frames * r.N
    nb = abi.pg_uv_prune_workspace_size(r.N, r.frames, M, Nv)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        abi.pg_uv_prune(r.params, r.n_gauss_dev, r.N, r.frames, r.C, M, Nv, K, None, uv, rank, keep, ws, nb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    passes = 4 + (max(1, (r.frames * M * Nv).bit_length()) + 7) // 8
    nbytes = n * (16 + 4 * 3 + 1) + passes * 20 * n      # read 4 channels, write uv/rank/keep; 20 B per item per pass
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"M": M, "N": Nv, "K": K, "ms": round(ms, 4), "gaussians": n, "kept": kept,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes": nbytes}}


def objective_leg(sc, r, atlas, target, tiling, steps, warmup, graph):
    """The full objective of the fitting step: the L1/SSIM blend (its kernel
    timed alone with events) and the step with it and both regularisers
    (weights 1e-4, the paper's)."""
    import torch
    stream = torch.cuda.current_stream()
    r.forward(atlas)
    r.loss_photo(target, LAMBDA_SSIM)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        r.loss_photo(target, LAMBDA_SSIM)
    e1.record(stream)
    torch.cuda.synchronize()
    lms = e0.elapsed_time(e1) / reps
    reg = {"s_max": S_MAX, "w_scale": 1e-4, "w_opacity": 1e-4}
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            r.step(atlas, target, lambda_ssim=LAMBDA_SSIM, reg=reg)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            r.step(atlas, target, lambda_ssim=LAMBDA_SSIM, reg=reg)
        torch.cuda.synchronize()
        run = g.replay
    else:
        def run():
            r.step(atlas, target, lambda_ssim=LAMBDA_SSIM, reg=reg)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    P = r.n_pixels
    fl = FLOP_PHOTO * 3 * P
    ach = fl / (lms / 1e3) / 1e12
    return {"lambda_ssim": LAMBDA_SSIM, "s_max": S_MAX, "w_scale": 1e-4, "w_opacity": 1e-4,
            "ms_per_step": round(ms, 4), "mpixels_per_s": round(P / ms / 1e3, 2), "loss": float(r.loss.item()),
            "photo_loss_ms": round(lms, 4),
            "photo_loss_roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                                    "flop_per_pixel_channel": FLOP_PHOTO}}


# FP64 operations of the flow-masking kernel: the projection chain per
# (Gaussian, view) (world and camera transforms, Sigma, Sigma_c, J, Sigma2D,
# det, lambda_max, mean, conic: about 300) and the quadratic form per tested
# pixel centre (9).
FLOP64_FMASK_RECORD = 300
FLOP64_FMASK_TEST = 9
PEAK_FP64_TFLOPS = 78.6


def flow_mask_leg(sc, r, atlas, reps=5):
    """Covariance-aware flow masking of the workload's Gaussians against seeded
    motion masks (discs over about 2 % of each view), timed with events on the
    stream it runs on; FP64-bound (the projection chain per Gaussian-view and
    the quadratic form per tested pixel)."""
    import torch

    import synth
    masks = torch.from_numpy(synth.flow_masks(sc, seed=44, coverage=0.02, mean_radius=0.02)).to("cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    dg, _ = r.flow_mask(atlas, masks, counters=cnt)
    torch.cuda.synchronize()
    tests = int(cnt.item())
    dyn = int(dg.sum().item())
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        r.flow_mask(atlas, masks)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps    # includes the fetch the call starts with (0.07 ms)
    n_gv = r.N * len(sc.cams)
    flops = FLOP64_FMASK_RECORD * n_gv + FLOP64_FMASK_TEST * tests
    ach = flops / (ms / 1e3) / 1e12
    return {"ms": round(ms, 4), "gaussian_views_per_s": round(n_gv / ms * 1e3, 1), "dynamic": dyn,
            "gaussians": r.N * sc.frames, "pixel_tests": tests,
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s (FP64)",
                         "frac": round(ach / PEAK_FP64_TFLOPS, 4)}}


def lpo_leg(sc, atlas, target, tiling, steps, warmup, graph):
    """The same step with the LPO fake quantiser after the fetch (16-bit
    position, 8-bit other channels), and the quantiser alone: its three
    kernels read each fetched value twice and write it once (12 bytes per
    value, HBM-bound), timed with events on the stream they run on."""
    import torch

    from paper_2602_23040_amd import _abi as abi
    from paper_2602_23040_amd.pipeline import Renderer

    dev = torch.device("cuda:0")
    bits = abi.lpo_bits(sc.C)
    r = Renderer(sc.occupancy, sc.frames, sc.sh_degree, sc.cams, tiling=tiling, batched=True, bg=sc.bg,
                 dynamic=sc.dynamic, device=dev, quant_bits=bits)
    r.forward(atlas)             # grows to the reported count after an overflow
    r.check_overflow = False
    stream = torch.cuda.current_stream()
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            r.step(atlas, target)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            r.step(atlas, target)
        torch.cuda.synchronize()
        run = g.replay
    else:
        def run():
            r.step(atlas, target)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert r.check()
    # the quantiser alone (re-quantising the proxy does the same work)
    reps = 20
    F, C, N = sc.frames, sc.C, r.N
    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for _ in range(reps):
        abi.pg_atlas_fake_quant(r.params, r.n_gauss_dev, N, F, C, bits, r.quant_range, None, r.quant_partial,
                                stream)
    q1.record(stream)
    torch.cuda.synchronize()
    qms = q0.elapsed_time(q1) / reps
    nbytes = 12 * F * C * N
    P = r.n_pixels
    r.close()
    gbs = nbytes / (qms / 1e3) / 1e9
    return {"bits": "16 (x, y, z), 8 (other channels)", "ms_per_step": round(ms, 4),
            "mpixels_per_s": round(P / ms / 1e3, 2), "fake_quant_ms": round(qms, 4),
            "fake_quant_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                    "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes": nbytes}}


def other_config(cfg, tiling, steps, warmup):
    """Batched (graph) and plain step time of another workload: fetch,
    projection, bin/sort, compositing, L1 against a second seeded Gaussian
    set, adjoint, and for the 2048^2 workload the sparse Adam update.
    tiling None: the autotuner picks it for this workload (cached)."""
    import numpy as np
    import torch

    import synth
    from paper_2602_23040_amd import autotune
    from paper_2602_23040_amd.pipeline import Renderer

    dev = torch.device("cuda:0")
    sc = synth.make_scene(cfg)
    tgt_sc = synth.make_scene(cfg, target=True)
    adam = cfg == 5
    atlas = torch.from_numpy(np.ascontiguousarray(sc.atlas).reshape(-1)).to(dev)
    tune_info = None
    if tiling is None:
        tiling, tune_info = autotune.choose(sc, atlas, device=dev)
        torch.cuda.empty_cache()
    tgt_atlas = torch.from_numpy(np.ascontiguousarray(tgt_sc.atlas).reshape(-1)).to(dev)
    del tgt_sc
    V, N = len(sc.cams), sc.n_gauss

    def make(batched, source, cap=None):
        r = Renderer(sc.occupancy, sc.frames, sc.sh_degree, sc.cams, tiling=tiling, batched=batched, bg=sc.bg,
                     dynamic=sc.dynamic, inst_capacity=cap, device=dev)
        r.forward(source)
        r.grow_capacity(1.3, headroom=True)     # Adam moves the Gaussians between replays
        r.check_overflow = False
        return r

    rt = make(True, tgt_atlas, 2 * N * V)
    rt.forward(tgt_atlas)
    torch.cuda.synchronize()
    target = rt.image.clone()
    rt.close()
    del rt, tgt_atlas
    torch.cuda.empty_cache()
    rb = make(True, atlas, 2 * N * V)
    work = atlas.clone()
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        rb.step(work, target, adam=adam)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rb.step(work, target, adam=adam)
    torch.cuda.synchronize()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert rb.check(), f"config {cfg}: instance capacity overflowed inside the timed region"
    n_inst = int(rb.sets[0].n_inst[0].item())
    P = rb.n_pixels
    adam_info = None
    if adam:
        # the sparse Adam kernel alone, on the state the last replay left: 28 algorithmic bytes per updated
        # element (read p, g, m, v; write p, m, v) plus 5 per texel (id and visibility lookups)
        n_vis = int(rb.visible.sum().item())
        elems = n_vis * sc.C
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        a0.record()
        for _ in range(reps):
            rb.adam_step(work)
        a1.record()
        torch.cuda.synchronize()
        adam_ms = a0.elapsed_time(a1) / reps
        alg = 28 * elems + 5 * sc.H * sc.W * sc.frames
        adam_info = {"ms": round(adam_ms, 4), "visible_gaussians": n_vis, "updated_elements": elems,
                     "roofline": {"bound": "hbm", "achieved": round(alg / adam_ms / 1e6, 1), "peak": 8000.0,
                                  "unit": "GB/s", "frac": round(alg / adam_ms / 1e6 / 8000.0, 4), "bytes": alg}}
    rb.close()
    del rb, graph
    torch.cuda.empty_cache()
    rp = make(False, atlas)
    work = atlas.clone()
    rp.step(work, target, adam=adam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        rp.step(work, target, adam=adam)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1e3 / 2
    rp.close()
    del rp
    torch.cuda.empty_cache()
    return {"config": cfg, "workload": sc.name, "views": V, "frames": sc.frames, "gaussians": N, "pixels": P,
            "instances": n_inst, "adam": adam, "steps": steps, "ms_per_step": round(ms, 3),
            "mpixels_per_s": round(P / ms / 1e3, 2), "gaussians_per_s": round(N * V / ms * 1e3, 1),
            "plain_ms_per_step": round(ms_plain, 3), "speedup_vs_plain": round(ms_plain / ms, 3),
            "tiling": "x".join(map(str, tiling)), "autotune": tune_info, "adam_kernel": adam_info}


def stage_times(r, atlas, target, reps=5):
    """Average duration of each entry point of the batched chain, timed with
    events on the stream the kernels are launched on."""
    import torch
    from paper_2602_23040_amd import _abi as abi

    s = r.sets[0]
    stream = torch.cuda.current_stream()
    calls = {
        "fetch": lambda: r.fetch(atlas),
        "project": lambda: abi.pg_project(s.handle, r.params, s.splats, s.bins, s.tiles, r.visible, stream),
        "bin_sort": lambda: abi.pg_bin_sort(s.handle, s.bins, s.tiles, s.cap, s.keys, s.values, s.ranges, s.order, s.inst_first,
                                            s.n_inst, s.overflow, s.ws, s.ws_bytes, stream),
        "render_fwd": lambda: abi.pg_render_fwd(s.handle, s.splats, s.values, s.ranges, s.order, r.bg, r.image, r.final_T,
                                                r.n_contrib, s.tile_entries, s.entries, None, stream),
        # the step's L1 path: the cotangent and the tiles' |image - target| sums inside the
        # compositing adjoint, then the loss value from those sums
        "render_bwd": lambda: abi.pg_render_bwd_l1(s.handle, s.splats, s.tiles, s.values, s.ranges, s.order,
                                                   s.inst_first, s.n_inst, s.cap, s.tile_entries, s.entries,
                                                   r.n_contrib, r.bg, r.final_T, r.image, target, 3 * r.n_pixels,
                                                   r.tile_loss, s.inst_grad, stream),
        "loss_l1": lambda: abi.pg_loss_l1_tiles(r.tile_loss, s.info.n_tiles, 3 * r.n_pixels, r.loss, stream),
        "project_bwd": lambda: abi.pg_project_bwd(s.handle, r.params, s.splats, s.bins, s.inst_first, s.n_inst,
                                                  s.cap, s.inst_grad, r.gauss_texel, r.dynamic, r.H, r.W, s.grad2d,
                                                  r.dL_datlas, 0, stream),
    }
    out = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        out[name] = a.elapsed_time(b) / reps
    return out


def cpu_baseline(sc, rb, target, budget_s):
    """FP64 oracle (as is) on the host cores over a bounded sample of views:
    forward + L1 (against a seeded random target) + adjoint per view until the
    time budget is used.  The GPU images of the same views are compared with
    the oracle's as a parity spot check."""
    import numpy as np

    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import explain

    sample = []
    t_total = 0.0
    img = rb.image.cpu().numpy()
    rng = np.random.default_rng(2024)
    beyond = unexplained = 0
    pix = 0
    for v in range(len(sc.cams)):
        t0 = time.perf_counter()
        fw = oracle.Forward(sc, views=[v])
        c = sc.cams[v]
        p0 = rb.pix_base[v]
        _, G = fw.loss({v: rng.uniform(0.0, 1.0, (3, c.height, c.width))})
        fw.backward(G)
        dt = time.perf_counter() - t0
        t_total += dt
        sample.append(v)
        pix += c.width * c.height
        gi = img[3 * p0:3 * (p0 + c.width * c.height)].reshape(3, c.height, c.width)
        _, unexp, nb = explain(fw, v, gi)
        beyond += nb
        unexplained += len(unexp)
        if t_total >= budget_s:
            break
    # the same work on one thread (the first view once more)
    cores = oracle.num_threads()
    c = sc.cams[0]
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        fw = oracle.Forward(sc, views=[0])
        _, G = fw.loss({0: rng.uniform(0.0, 1.0, (3, c.height, c.width))})
        fw.backward(G)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": round(pix / t_total / 1e6, 4), "unit": "Mpixels/s", "cores": cores,
            "kind": "oracle",
            "sample": f"views {sample} of the same workload (fwd + L1 + adjoint, FP64), {t_total:.1f} s",
            "single_thread": {"value": round(c.width * c.height / t1 / 1e6, 4), "unit": "Mpixels/s",
                              "sample": f"view 0, {t1:.1f} s"},
            "host": {"cpu": host_cpu(), "nproc": os.cpu_count()},
            "parity_sample": {"pixels": pix, "beyond_1e-4": beyond, "unexplained": unexplained}}


if __name__ == "__main__":
    main()
