"""ctypes binding of ``include/packuv_gs.h`` -- argument marshalling only.

Every function here has the name of the C entry point it calls and accepts
torch tensors (their device pointers are passed) or plain integers.  No
computation happens on this side; a missing library is an error, never a
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpackuvgs.so")

PG_OK = 0
STATUS_NAMES = {0: "PG_OK", -1: "PG_ERR_INVALID_ARG", -2: "PG_ERR_UNSUPPORTED_DEVICE", -3: "PG_ERR_CAPACITY",
                -4: "PG_ERR_HIP", -5: "PG_ERR_WORKSPACE"}

SPLAT_BYTES = 48
SLOT_WORDS = 10             # words of one per-instance gradient slot (nine sums and the generation tag)
BIN_BYTES = 16
QUANT_BLOCKS = 256          # PG_QUANT_BLOCKS: the fake quantiser's workspace is 2 * QUANT_BLOCKS * C floats
REG_BLOCKS = 256            # PG_REG_BLOCKS: the regularisers' workspace is 3 * REG_BLOCKS + 1 doubles


class PGError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pg_camera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
                ("frame", C.c_int32), ("reserved", C.c_int32)]


class pg_tiling(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("lds_batch", C.c_int32), ("reserved", C.c_int32)]


class pg_views_info(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("frames", C.c_int32), ("n_gauss", C.c_int64), ("sh_degree", C.c_int32),
                ("channels", C.c_int32), ("n_gv", C.c_int64), ("n_tiles", C.c_int64), ("n_pixels", C.c_int64),
                ("key_bits", C.c_int32), ("sort_passes", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("lds_batch", C.c_int32), ("reserved", C.c_int32)]


PLAN_FIELDS = ["params", "gauss_texel", "texel_gauss", "n_gauss", "fetch_ws", "visible", "splats", "bins",
               "tile_sets", "keys", "values", "tile_ranges", "tile_order", "inst_first", "n_inst", "overflow",
               "sort_ws", "inst_grad", "image", "final_T", "n_contrib", "tile_entries", "entries", "dL_dimage",
               "grad2d", "dL_datlas", "total"]


class pg_plan(C.Structure):
    _fields_ = [(f, C.c_size_t) for f in PLAN_FIELDS]


assert C.sizeof(pg_camera) == 144 and C.sizeof(pg_views_info) == 72 and C.sizeof(pg_plan) == 8 * 27

_lib = None

# name -> (restype, argtypes); p = pointer-sized integer (device or host address)
_p, _i32, _i64, _u64, _f32, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float, C.c_size_t
SIGNATURES = {
    "pg_init": (_i32, [_i32]),
    "pg_last_error": (C.c_char_p, []),
    "pg_views_create": (_i32, [C.POINTER(pg_camera), _i32, _i32, _i64, _i32, pg_tiling, C.POINTER(_p)]),
    "pg_views_destroy": (_i32, [_p]),
    "pg_views_get_info": (_i32, [_p, C.POINTER(pg_views_info)]),
    "pg_views_offsets": (_i32, [_p, _p, _p]),
    "pg_fetch_workspace_size": (_i32, [_i32, _i32, C.POINTER(_sz)]),
    "pg_sort_workspace_size": (_i32, [_p, _i64, C.POINTER(_sz)]),
    "pg_atlas_fetch": (_i32, [_p, _p, _i32, _i32, _i32, _i32, _i64, _p, _p, _p, _p, _p, _sz, _p]),
    "pg_atlas_fetch_noalloc": (_i32, [_p, _p, _i32, _i32, _i32, _i32, _i64, _p, _p, _p, _p, _p]),
    "pg_atlas_fake_quant": (_i32, [_p, _p, _i64, _i32, _i32, _p, _p, _p, _p, _p]),
    "pg_project": (_i32, [_p, _p, _p, _p, _p, _p, _p]),
    "pg_flow_mask": (_i32, [_p, _p, _p, _p, _p, _p, _i32, _i32, _p, _p, _p]),
    "pg_bin_sort": (_i32, [_p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "pg_render_fwd": (_i32, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]),
    "pg_render_bwd": (_i32, [_p, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p]),
    "pg_render_bwd_l1": (_i32, [_p, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _p,
                                _p]),
    "pg_loss_l1_tiles": (_i32, [_p, _i64, _i64, _p, _p]),
    "pg_project_bwd": (_i32, [_p, _p, _p, _p, _p, _p, _i64, _p, _p, _p, _i32, _i32, _p, _p, _i32, _p]),
    "pg_backward": (_i32, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i32,
                           _i32, _p, _p, _i32, _p]),
    "pg_status_check": (_i32, [_p, _p, _p, _p]),
    "pg_workspace_query": (_i32, [_p, _i32, _i32, _i64, C.POINTER(pg_plan)]),
    "pg_loss_l1": (_i32, [_p, _p, _i64, _p, _p, _p, _p]),
    "pg_photo_workspace_size": (_i32, [_p, C.POINTER(_sz)]),
    "pg_uv_prune_workspace_size": (_i32, [_i64, _i32, _i32, _i32, C.POINTER(_sz)]),
    "pg_uv_prune": (_i32, [_p, _p, _i64, _i32, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p, _sz, _p]),
    "pg_loss_regularisers": (_i32, [_p, _p, _i64, _i32, _i32, _p, _i32, _i32, _p, _f32, _f32, _f32, _p, _p, _p, _p]),
    "pg_loss_photo": (_i32, [_p, _p, _p, _f32, _p, _p, _p, _sz, _p]),
    "pg_adam_step": (_i32, [_p, _p, _p, _p, _p, _p, _i64, _i32, _i32, _i32, _i32, _f32, _f32, _f32, _f32, _i32, _p,
                            _p]),
}


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python paper_2602_23040_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, C.c_void_p):
        return x.value
    raise TypeError(f"cannot pass {type(x)} as a pointer")


def _check(status: int, where: str):
    if status != PG_OK:
        msg = lib().pg_last_error()
        raise PGError(status, where, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def make_camera(cam) -> pg_camera:
    import numpy as np
    c = pg_camera()
    R = np.asarray(cam.R, np.float64).reshape(-1)
    t = np.asarray(cam.t, np.float64).reshape(-1)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height, c.frame, c.reserved = int(cam.width), int(cam.height), int(cam.frame), 0
    return c


def make_tiling(tile_w=16, tile_h=16, lds_batch=256) -> pg_tiling:
    return pg_tiling(int(tile_w), int(tile_h), int(lds_batch), 0)


# --------------------------------------------------------------------------- entry points

def pg_init(device: int = 0):
    _check(lib().pg_init(int(device)), "pg_init")


def pg_last_error() -> str:
    m = lib().pg_last_error()
    return m.decode() if m else ""


def pg_views_create(cams, frames: int, n_gauss: int, sh_degree: int, tiling: pg_tiling):
    arr = (pg_camera * len(cams))(*[make_camera(c) for c in cams])
    out = C.c_void_p()
    _check(lib().pg_views_create(arr, len(cams), int(frames), int(n_gauss), int(sh_degree), tiling, C.byref(out)),
           "pg_views_create")
    return out.value


def pg_views_destroy(views):
    _check(lib().pg_views_destroy(views), "pg_views_destroy")


def pg_views_get_info(views) -> pg_views_info:
    info = pg_views_info()
    _check(lib().pg_views_get_info(views, C.byref(info)), "pg_views_get_info")
    return info


def pg_views_offsets(views, n_views: int):
    tb = (C.c_int64 * (n_views + 1))()
    pb = (C.c_int64 * (n_views + 1))()
    _check(lib().pg_views_offsets(views, C.addressof(tb), C.addressof(pb)), "pg_views_offsets")
    return list(tb), list(pb)


def pg_fetch_workspace_size(H: int, W: int) -> int:
    n = C.c_size_t()
    _check(lib().pg_fetch_workspace_size(int(H), int(W), C.byref(n)), "pg_fetch_workspace_size")
    return n.value


def pg_sort_workspace_size(views, inst_capacity: int) -> int:
    n = C.c_size_t()
    _check(lib().pg_sort_workspace_size(views, int(inst_capacity), C.byref(n)), "pg_sort_workspace_size")
    return n.value


def pg_atlas_fetch(atlas, occupancy, frames, channels, H, W, n_cap, gauss_texel, texel_gauss, params, n_gauss_dev,
                   ws, ws_bytes, stream=None):
    _check(lib().pg_atlas_fetch(_ptr(atlas), _ptr(occupancy), int(frames), int(channels), int(H), int(W), int(n_cap),
                                _ptr(gauss_texel), _ptr(texel_gauss), _ptr(params), _ptr(n_gauss_dev), _ptr(ws),
                                int(ws_bytes), _stream(stream)), "pg_atlas_fetch")


FETCH_NOALLOC_MAX_TEXELS = 1 << 26          # PG_FETCH_NOALLOC_MAX_TEXELS
FETCH_NOALLOC_SCRATCH_BYTES = 256 * 1024     # PG_FETCH_NOALLOC_SCRATCH_BYTES


def pg_atlas_fetch_noalloc(atlas, occupancy, frames, channels, H, W, n_cap, gauss_texel, texel_gauss, params,
                           n_gauss_dev, stream=None):
    _check(lib().pg_atlas_fetch_noalloc(_ptr(atlas), _ptr(occupancy), int(frames), int(channels), int(H), int(W),
                                        int(n_cap), _ptr(gauss_texel), _ptr(texel_gauss), _ptr(params),
                                        _ptr(n_gauss_dev), _stream(stream)), "pg_atlas_fetch_noalloc")


def pg_atlas_fake_quant(params, n_gauss_dev, n_cap, frames, channels, bits, range_out, codes, partial, stream=None):
    """LPO proxy in place; `bits` is a host sequence of per-channel widths."""
    b = (C.c_int32 * int(channels))(*[int(x) for x in bits])
    _check(lib().pg_atlas_fake_quant(_ptr(params), _ptr(n_gauss_dev), int(n_cap), int(frames), int(channels),
                                     C.cast(b, _p), _ptr(range_out), _ptr(codes), _ptr(partial), _stream(stream)),
           "pg_atlas_fake_quant")


def pg_flow_mask(views, params, flow_masks, tile_motion, dyn_gauss, texel_gauss, H, W, dyn_texel, counters,
                 stream=None):
    _check(lib().pg_flow_mask(views, _ptr(params), _ptr(flow_masks), _ptr(tile_motion), _ptr(dyn_gauss),
                              _ptr(texel_gauss), int(H),
                              int(W), _ptr(dyn_texel), _ptr(counters), _stream(stream)), "pg_flow_mask")


def lpo_bits(channels):
    """The paper's LPO widths: 16 bits for the position (x, y, z), 8 for every
    other channel (log-scale, quaternion, logit-opacity, SH)."""
    return [16, 16, 16] + [8] * (int(channels) - 3)


def pg_project(views, params, splats, bins, tiles, visible, stream=None):
    _check(lib().pg_project(views, _ptr(params), _ptr(splats), _ptr(bins), _ptr(tiles), _ptr(visible),
                            _stream(stream)), "pg_project")


def pg_bin_sort(views, bins, tiles, inst_capacity, keys, values, tile_ranges, tile_order, inst_first, n_inst_dev,
                overflow_dev, ws, ws_bytes, stream=None):
    _check(lib().pg_bin_sort(views, _ptr(bins), _ptr(tiles), int(inst_capacity), _ptr(keys), _ptr(values), _ptr(tile_ranges),
                             _ptr(tile_order), _ptr(inst_first), _ptr(n_inst_dev), _ptr(overflow_dev), _ptr(ws),
                             int(ws_bytes),
                             _stream(stream)), "pg_bin_sort")


def pg_render_fwd(views, splats, values, tile_ranges, tile_order, bg, image, final_T, n_contrib, tile_entries, entries,
                  counters=None, stream=None):
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    _check(lib().pg_render_fwd(views, _ptr(splats), _ptr(values), _ptr(tile_ranges), _ptr(tile_order),
                               C.addressof(bgv), _ptr(image),
                               _ptr(final_T), _ptr(n_contrib), _ptr(tile_entries), _ptr(entries), _ptr(counters),
                               _stream(stream)), "pg_render_fwd")


def pg_render_bwd(views, splats, tiles, values, tile_ranges, tile_order, inst_first, n_inst_dev, inst_capacity,
                  tile_entries, entries, n_contrib, bg, final_T, dL_dimage, inst_grad, stream=None):
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    _check(lib().pg_render_bwd(views, _ptr(splats), _ptr(tiles), _ptr(values), _ptr(tile_ranges), _ptr(tile_order),
                               _ptr(inst_first),
                               _ptr(n_inst_dev), int(inst_capacity), _ptr(tile_entries), _ptr(entries),
                               _ptr(n_contrib), C.addressof(bgv), _ptr(final_T), _ptr(dL_dimage), _ptr(inst_grad),
                               _stream(stream)), "pg_render_bwd")


def pg_render_bwd_l1(views, splats, tiles, values, tile_ranges, tile_order, inst_first, n_inst_dev, inst_capacity,
                     tile_entries, entries, n_contrib, bg, final_T, image, target, n, tile_loss, inst_grad,
                     stream=None):
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    _check(lib().pg_render_bwd_l1(views, _ptr(splats), _ptr(tiles), _ptr(values), _ptr(tile_ranges),
                                  _ptr(tile_order), _ptr(inst_first), _ptr(n_inst_dev), int(inst_capacity),
                                  _ptr(tile_entries), _ptr(entries), _ptr(n_contrib), C.addressof(bgv),
                                  _ptr(final_T), _ptr(image), _ptr(target), int(n), _ptr(tile_loss),
                                  _ptr(inst_grad), _stream(stream)), "pg_render_bwd_l1")


def pg_loss_l1_tiles(tile_loss, n_tiles, n, loss_dev, stream=None):
    _check(lib().pg_loss_l1_tiles(_ptr(tile_loss), int(n_tiles), int(n), _ptr(loss_dev), _stream(stream)),
           "pg_loss_l1_tiles")


def pg_project_bwd(views, params, splats, bins, inst_first, n_inst_dev, inst_capacity, inst_grad, gauss_texel,
                   dynamic_mask, H, W, grad2d, dL_datlas, accumulate, stream=None):
    _check(lib().pg_project_bwd(views, _ptr(params), _ptr(splats), _ptr(bins), _ptr(inst_first), _ptr(n_inst_dev),
                                int(inst_capacity), _ptr(inst_grad), _ptr(gauss_texel),
                                _ptr(dynamic_mask), int(H), int(W), _ptr(grad2d), _ptr(dL_datlas), int(accumulate),
                                _stream(stream)), "pg_project_bwd")


def pg_backward(views, params, splats, bins, tiles, values, tile_ranges, tile_order, inst_first, n_inst_dev,
                inst_capacity, tile_entries, entries, n_contrib, bg, final_T, dL_dimage, inst_grad, gauss_texel,
                dynamic_mask, H, W, grad2d, dL_datlas, accumulate, stream=None):
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    _check(lib().pg_backward(views, _ptr(params), _ptr(splats), _ptr(bins), _ptr(tiles), _ptr(values),
                             _ptr(tile_ranges), _ptr(tile_order), _ptr(inst_first), _ptr(n_inst_dev),
                             int(inst_capacity), _ptr(tile_entries), _ptr(entries), _ptr(n_contrib), C.addressof(bgv),
                             _ptr(final_T), _ptr(dL_dimage), _ptr(inst_grad), _ptr(gauss_texel), _ptr(dynamic_mask),
                             int(H), int(W), _ptr(grad2d), _ptr(dL_datlas), int(accumulate), _stream(stream)),
           "pg_backward")


PG_ERR_CAPACITY = -3


def pg_status_check(overflow_dev, n_inst_dev, stream=None):
    """(overflowed, needed capacity); synchronises the stream.  Errors other
    than PG_ERR_CAPACITY raise."""
    need = C.c_int64()
    st = lib().pg_status_check(_ptr(overflow_dev), _ptr(n_inst_dev), C.byref(need), _stream(stream))
    if st not in (PG_OK, PG_ERR_CAPACITY):
        _check(st, "pg_status_check")
    return st == PG_ERR_CAPACITY, int(need.value)


def pg_workspace_query(views, H, W, inst_capacity) -> dict:
    plan = pg_plan()
    _check(lib().pg_workspace_query(views, int(H), int(W), int(inst_capacity), C.byref(plan)), "pg_workspace_query")
    return {f: int(getattr(plan, f)) for f in PLAN_FIELDS}


def pg_loss_l1(image, target, n, dL_dimage, partial, loss_dev, stream=None):
    _check(lib().pg_loss_l1(_ptr(image), _ptr(target), int(n), _ptr(dL_dimage), _ptr(partial), _ptr(loss_dev),
                            _stream(stream)), "pg_loss_l1")


def pg_photo_workspace_size(views) -> int:
    n = C.c_size_t()
    _check(lib().pg_photo_workspace_size(views, C.byref(n)), "pg_photo_workspace_size")
    return n.value


def pg_loss_photo(views, image, target, lambda_ssim, dL_dimage, loss_dev, ws, ws_bytes, stream=None):
    _check(lib().pg_loss_photo(views, _ptr(image), _ptr(target), float(lambda_ssim), _ptr(dL_dimage), _ptr(loss_dev),
                               _ptr(ws), int(ws_bytes), _stream(stream)), "pg_loss_photo")


def pg_loss_regularisers(params, n_gauss_dev, n_cap, frames, channels, gauss_texel, H, W, dyn_gauss, s_max,
                         w_scale, w_opacity, dL_datlas, reg_loss, partial, stream=None):
    _check(lib().pg_loss_regularisers(_ptr(params), _ptr(n_gauss_dev), int(n_cap), int(frames), int(channels),
                                      _ptr(gauss_texel), int(H), int(W), _ptr(dyn_gauss), float(s_max),
                                      float(w_scale), float(w_opacity), _ptr(dL_datlas), _ptr(reg_loss),
                                      _ptr(partial), _stream(stream)), "pg_loss_regularisers")


def pg_uv_prune_workspace_size(n_cap, frames, M, Nv) -> int:
    n = C.c_size_t()
    _check(lib().pg_uv_prune_workspace_size(int(n_cap), int(frames), int(M), int(Nv), C.byref(n)),
           "pg_uv_prune_workspace_size")
    return n.value


def pg_uv_prune(params, n_gauss_dev, n_cap, frames, channels, M, Nv, K, expected_uv, uv, rank, keep, ws, ws_bytes,
                stream=None):
    _check(lib().pg_uv_prune(_ptr(params), _ptr(n_gauss_dev), int(n_cap), int(frames), int(channels), int(M), int(Nv),
                             int(K), _ptr(expected_uv), _ptr(uv), _ptr(rank), _ptr(keep), _ptr(ws), int(ws_bytes),
                             _stream(stream)), "pg_uv_prune")


def pg_adam_step(atlas, grad, m, v, visible, texel_gauss, n_gauss, frames, channels, H, W, lr, beta1, beta2, eps,
                 step, step_dev=None, stream=None):
    _check(lib().pg_adam_step(_ptr(atlas), _ptr(grad), _ptr(m), _ptr(v), _ptr(visible), _ptr(texel_gauss),
                              int(n_gauss), int(frames), int(channels), int(H), int(W), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), _ptr(step_dev), _stream(stream)), "pg_adam_step")
