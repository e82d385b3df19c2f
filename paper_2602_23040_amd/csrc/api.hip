// C ABI of the library: argument validation, the device-resident view
// table, and the entry points that enqueue the kernels of the other
// translation units.  Every check that can be made on the host is made
// before anything is enqueued.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pg_internal.h"

namespace pg {

namespace {
thread_local std::string g_error;

pg_status invalid(const std::string& msg) {
    g_error = msg;
    return PG_ERR_INVALID_ARG;
}

bool tiling_ok(const pg_tiling& t) {
    const bool shape = (t.tile_w == 16 && t.tile_h == 16) || (t.tile_w == 8 && t.tile_h == 32) ||
                       (t.tile_w == 32 && t.tile_h == 8);
    const bool batch = t.lds_batch == 64 || t.lds_batch == 128 || t.lds_batch == 256;
    return shape && batch && t.reserved == 0;
}

#define PG_CHECK_HIP(expr, what)                          \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, what);  \
    } while (0)

// Workspace of pg_atlas_fetch_noalloc: a fixed array in device memory, one
// copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel or a copy (in host code it is a stand-in, not a device
// address); it uses the per-device address that hipGetSymbolAddress returns.
constexpr size_t kFetchScratchBytes = PG_FETCH_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kFetchScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of `scratch` (looked up once per
// device, with that device current).
pg_status scratch_for_current_device(void** out) {
    int dev = -1;
    PG_CHECK_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        g_error = "device index beyond the library's per-device table";
        return PG_ERR_UNSUPPORTED_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        PG_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) {
            g_error = "hipGetSymbolAddress(scratch) returned a null address";
            return PG_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

pg_status hip_fail(hipError_t e, const char* what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return PG_ERR_HIP;
}

}  // namespace pg

using namespace pg;

extern "C" {

const char* pg_last_error(void) { return g_error.c_str(); }

pg_status pg_init(int32_t device) {
    g_error.clear();
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        set_error("no HIP device available");
        return PG_ERR_UNSUPPORTED_DEVICE;
    }
    if (device < 0 || device >= n) return invalid("device index out of range");
    PG_CHECK_HIP(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    PG_CHECK_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error(std::string("unsupported device architecture ") + prop.gcnArchName + " (needs gfx950)");
        return PG_ERR_UNSUPPORTED_DEVICE;
    }
    void* ws = nullptr;
    return scratch_for_current_device(&ws);
}

pg_status pg_views_create(const pg_camera* cams, int32_t n_views, int32_t frames, int64_t n_gauss,
                          int32_t sh_degree, pg_tiling tiling, pg_views** out) {
    g_error.clear();
    if (!out) return invalid("out is null");
    *out = nullptr;
    if (!cams) return invalid("cams is null");
    if (n_views < 1 || n_views > kMaxViews) return invalid("n_views must be in [1, 65536]");
    if (frames < 1 || frames > 65535) return invalid("frames must be in [1, 65535]");
    if (n_gauss < 0) return invalid("n_gauss must be >= 0");
    if (sh_degree < 0 || sh_degree > 3) return invalid("sh_degree must be in [0, 3]");
    if (!tiling_ok(tiling))
        return invalid("tiling must be 16x16, 8x32 or 32x8 with lds_batch 64, 128 or 256 (reserved = 0)");
    if ((int64_t)n_views * n_gauss > INT32_MAX) return invalid("n_views * n_gauss exceeds 2^31 - 1");
    if (n_gauss > ((int64_t)1 << 28)) return invalid("n_gauss exceeds 2^28");
    std::vector<ViewDev> hv(n_views);
    std::vector<int64_t> tb(n_views + 1), pb(n_views + 1), sb(n_views);
    int64_t tiles = 0, pixels = 0, sblocks = 0;
    for (int32_t v = 0; v < n_views; v++) {
        const pg_camera& c = cams[v];
        if (!(c.fx > 0.0) || !(c.fy > 0.0) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
            return invalid("camera " + std::to_string(v) + ": fx and fy must be finite and > 0");
        if (c.width < 1 || c.height < 1 || c.width > 32767 * 8 || c.height > 32767 * 8)
            return invalid("camera " + std::to_string(v) + ": width and height must be in [1, 262136]");
        if (c.frame < 0 || c.frame >= frames)
            return invalid("camera " + std::to_string(v) + ": frame out of range");
        if (c.reserved != 0) return invalid("camera " + std::to_string(v) + ": reserved must be 0");
        for (int k = 0; k < 9; k++)
            if (!std::isfinite(c.R[k])) return invalid("camera " + std::to_string(v) + ": R not finite");
        for (int k = 0; k < 3; k++)
            if (!std::isfinite(c.t[k])) return invalid("camera " + std::to_string(v) + ": t not finite");
        ViewDev& d = hv[v];
        std::memset(&d, 0, sizeof d);
        std::memcpy(d.R, c.R, sizeof d.R);
        std::memcpy(d.t, c.t, sizeof d.t);
        d.fx = c.fx;
        d.fy = c.fy;
        d.cx = c.cx;
        d.cy = c.cy;
        for (int k = 0; k < 3; k++) d.cw[k] = -((c.R[k] * c.t[0] + c.R[3 + k] * c.t[1]) + c.R[6 + k] * c.t[2]);
        for (int k = 0; k < 9; k++) d.Rf[k] = (float)d.R[k];
        for (int k = 0; k < 3; k++) {
            d.tf[k] = (float)d.t[k];
            d.cwf[k] = (float)d.cw[k];
        }
        d.fxf = (float)d.fx;
        d.fyf = (float)d.fy;
        d.W = c.width;
        d.H = c.height;
        d.TX = (c.width + tiling.tile_w - 1) / tiling.tile_w;
        d.TY = (c.height + tiling.tile_h - 1) / tiling.tile_h;
        d.frame = c.frame;
        d.tile_base = tiles;
        d.pix_base = pixels;
        tb[v] = tiles;
        pb[v] = pixels;
        sb[v] = sblocks;
        sblocks += (int64_t)((c.width + 31) / 32) * ((c.height + 31) / 32);
        tiles += (int64_t)d.TX * d.TY;
        pixels += (int64_t)c.width * c.height;
    }
    tb[n_views] = tiles;
    pb[n_views] = pixels;
    if (tiles > INT32_MAX) return invalid("total tile count exceeds 2^31 - 1");
    std::vector<int32_t> fv(frames + 1, 0), order;
    for (int32_t f = 0; f < frames; f++) {
        fv[f] = (int32_t)order.size();
        for (int32_t v = 0; v < n_views; v++)
            if (cams[v].frame == f) order.push_back(v);
    }
    fv[frames] = (int32_t)order.size();
    int tile_bits = 1;
    while ((int64_t(1) << tile_bits) < tiles) tile_bits++;

    pg_views* p = new pg_views();
    p->n_views = n_views;
    p->frames = frames;
    p->sh_degree = sh_degree;
    p->channels = 11 + 3 * (sh_degree + 1) * (sh_degree + 1);
    p->n_gauss = n_gauss;
    p->tiling = tiling;
    p->n_gv = (int64_t)n_views * n_gauss;
    p->n_tiles = tiles;
    p->n_pixels = pixels;
    p->key_bits = tile_bits;
    p->sort_passes = (32 + 7) / 8 + (tile_bits + 7) / 8;   // record (depth) passes + instance (tile) passes
    p->n_ssim_blocks = sblocks;
    p->h_tile_base = new int64_t[n_views + 1];
    p->h_pix_base = new int64_t[n_views + 1];
    std::memcpy(p->h_tile_base, tb.data(), sizeof(int64_t) * (n_views + 1));
    std::memcpy(p->h_pix_base, pb.data(), sizeof(int64_t) * (n_views + 1));
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->d_views, sizeof(ViewDev) * n_views);
    if (e == hipSuccess) e = hipMalloc(&p->d_frame_views, sizeof(int32_t) * (frames + 1));
    if (e == hipSuccess) e = hipMalloc(&p->d_view_order, sizeof(int32_t) * n_views);
    if (e == hipSuccess) e = hipMalloc(&p->d_ssim_base, sizeof(int64_t) * n_views);
    if (e == hipSuccess) e = hipMemcpy(p->d_ssim_base, sb.data(), sizeof(int64_t) * n_views, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_views, hv.data(), sizeof(ViewDev) * n_views, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_frame_views, fv.data(), sizeof(int32_t) * (frames + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_view_order, order.data(), sizeof(int32_t) * n_views, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pg_views_destroy(p);
        return hip_fail(e, "pg_views_create");
    }
    *out = p;
    return PG_OK;
}

pg_status pg_views_destroy(pg_views* v) {
    if (!v) return PG_OK;
    hipError_t e = hipSuccess;
    for (void* d : {(void*)v->d_views, (void*)v->d_frame_views, (void*)v->d_view_order, (void*)v->d_ssim_base}) {
        if (!d) continue;
        const hipError_t r = hipFree(d);
        if (e == hipSuccess) e = r;      // free everything, report the first failure
    }
    delete[] v->h_tile_base;
    delete[] v->h_pix_base;
    delete v;
    return e == hipSuccess ? PG_OK : hip_fail(e, "pg_views_destroy");
}

pg_status pg_views_get_info(const pg_views* v, pg_views_info* info) {
    if (!v || !info) return invalid("null argument");
    std::memset(info, 0, sizeof *info);
    info->n_views = v->n_views;
    info->frames = v->frames;
    info->n_gauss = v->n_gauss;
    info->sh_degree = v->sh_degree;
    info->channels = v->channels;
    info->n_gv = v->n_gv;
    info->n_tiles = v->n_tiles;
    info->n_pixels = v->n_pixels;
    info->key_bits = v->key_bits;
    info->sort_passes = v->sort_passes;
    info->tile_w = v->tiling.tile_w;
    info->tile_h = v->tiling.tile_h;
    info->lds_batch = v->tiling.lds_batch;
    return PG_OK;
}

pg_status pg_views_offsets(const pg_views* v, int64_t* tile_base, int64_t* pixel_base) {
    if (!v || !tile_base || !pixel_base) return invalid("null argument");
    std::memcpy(tile_base, v->h_tile_base, sizeof(int64_t) * (v->n_views + 1));
    std::memcpy(pixel_base, v->h_pix_base, sizeof(int64_t) * (v->n_views + 1));
    return PG_OK;
}

pg_status pg_fetch_workspace_size(int32_t H, int32_t W, size_t* bytes) {
    if (!bytes) return invalid("bytes is null");
    if (H < 1 || W < 1) return invalid("H and W must be >= 1");
    *bytes = fetch_ws_bytes(H, W);
    return PG_OK;
}

pg_status pg_sort_workspace_size(const pg_views* v, int64_t cap, size_t* bytes) {
    if (!v || !bytes) return invalid("null argument");
    if (cap < 0 || cap > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    *bytes = sort_ws_bytes(v, cap);
    return PG_OK;
}

pg_status pg_atlas_fetch(const float* atlas, const uint8_t* occupancy, int32_t frames, int32_t channels, int32_t H,
                         int32_t W, int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss, float* params,
                         int64_t* n_gauss_dev, void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    if (!atlas || !occupancy || !texel_gauss || !n_gauss_dev || !ws) return invalid("null pointer argument");
    if (n_cap > 0 && (!gauss_texel || !params)) return invalid("gauss_texel / params null with n_cap > 0");
    if (frames < 1 || channels < 1 || H < 1 || W < 1 || n_cap < 0) return invalid("bad sizes");
    if ((int64_t)H * W > INT32_MAX) return invalid("H * W exceeds 2^31 - 1");
    if (ws_bytes < fetch_ws_bytes(H, W)) {
        set_error("fetch workspace too small");
        return PG_ERR_WORKSPACE;
    }
    PG_CHECK_HIP(launch_fetch(atlas, occupancy, frames, channels, H, W, n_cap, gauss_texel, texel_gauss, params,
                              n_gauss_dev, ws, (hipStream_t)stream),
                 "pg_atlas_fetch");
    return PG_OK;
}

pg_status pg_atlas_fetch_noalloc(const float* atlas, const uint8_t* occupancy, int32_t frames, int32_t channels,
                                 int32_t H, int32_t W, int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss,
                                 float* params, int64_t* n_gauss_dev, void* stream) {
    g_error.clear();
    if (!atlas || !occupancy || !texel_gauss || !n_gauss_dev) return invalid("null pointer argument");
    if (n_cap > 0 && (!gauss_texel || !params)) return invalid("gauss_texel / params null with n_cap > 0");
    if (frames < 1 || channels < 1 || H < 1 || W < 1 || n_cap < 0) return invalid("bad sizes");
    if ((int64_t)H * W > INT32_MAX) return invalid("H * W exceeds 2^31 - 1");
    if ((int64_t)H * W > PG_FETCH_NOALLOC_MAX_TEXELS || fetch_ws_bytes(H, W) > kFetchScratchBytes) {
        set_error("atlas of " + std::to_string((int64_t)H * W) + " texels is larger than the " +
                  std::to_string((int64_t)PG_FETCH_NOALLOC_MAX_TEXELS) +
                  " that the library's fixed scratch serves; use pg_atlas_fetch with a workspace");
        return PG_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    const pg_status st = scratch_for_current_device(&ws);
    if (st != PG_OK) return st;
    // Every word of the workspace that the kernels read is written earlier in
    // the same call (block counts, then their scan), so nothing is cleared.
    PG_CHECK_HIP(launch_fetch(atlas, occupancy, frames, channels, H, W, n_cap, gauss_texel, texel_gauss, params,
                              n_gauss_dev, ws, (hipStream_t)stream),
                 "pg_atlas_fetch_noalloc");
    return PG_OK;
}

pg_status pg_project(const pg_views* v, const float* params, pg_splat* splats, pg_bin* bins, pg_tile_set* tiles,
                     uint8_t* visible, void* stream) {
    g_error.clear();
    if (!v) return invalid("views is null");
    if (v->n_gv > 0 && (!params || !splats || !bins || !tiles || !visible)) return invalid("null pointer argument");
    PG_CHECK_HIP(launch_project(v, params, splats, bins, tiles, visible, (hipStream_t)stream), "pg_project");
    return PG_OK;
}

pg_status pg_bin_sort(const pg_views* v, const pg_bin* bins, const pg_tile_set* tiles, int64_t cap, uint32_t* keys,
                      int32_t* values,
                      int32_t* tile_ranges, int32_t* tile_order, int32_t* inst_first, int64_t* n_inst_dev, int32_t* overflow_dev,
                      void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    if (!v) return invalid("views is null");
    if (!tile_ranges || !n_inst_dev || !overflow_dev || !ws) return invalid("null pointer argument");
    if (v->n_gv > 0 && (!bins || !tiles || !inst_first)) return invalid("bins / tiles / inst_first is null");
    if (cap < 0 || cap > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    if (cap > 0 && (!keys || !values)) return invalid("keys / values null with inst_capacity > 0");
    if (ws_bytes < sort_ws_bytes(v, cap)) {
        set_error("sort workspace too small");
        return PG_ERR_WORKSPACE;
    }
    PG_CHECK_HIP(launch_bin_sort(v, bins, tiles, cap, keys, values, tile_ranges, tile_order, inst_first, n_inst_dev, overflow_dev,
                                 ws, (hipStream_t)stream),
                 "pg_bin_sort");
    return PG_OK;
}

pg_status pg_render_fwd(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* tile_ranges,
                        const int32_t* tile_order, const float* bg, float* image, float* final_T, int32_t* n_contrib, int32_t* tile_entries,
                        uint32_t* entries, uint64_t* counters, void* stream) {
    g_error.clear();
    if (!v || !bg) return invalid("null argument");
    if (!image || !final_T || !n_contrib || !tile_ranges || !tile_entries) return invalid("null pointer argument");
    if (v->n_gv > 0 && (!splats || !values || !entries)) return invalid("null pointer argument");
    PG_CHECK_HIP(launch_render_fwd(v, splats, values, tile_ranges, tile_order, bg, image, final_T, n_contrib, tile_entries,
                                   entries, counters, (hipStream_t)stream),
                 "pg_render_fwd");
    return PG_OK;
}

pg_status pg_render_bwd(const pg_views* v, const pg_splat* splats, const pg_tile_set* tiles,
                        const int32_t* values, const int32_t* tile_ranges, const int32_t* tile_order,
                        const int32_t* inst_first, const int64_t* n_inst_dev,
                        int64_t inst_capacity, const int32_t* tile_entries, const uint32_t* entries,
                        const int32_t* n_contrib, const float* bg, const float* final_T, const float* dL_dimage,
                        float* inst_grad, void* stream) {
    g_error.clear();
    if (!v || !bg) return invalid("null argument");
    if (!tile_ranges || !tile_entries || !n_contrib || !final_T || !dL_dimage || !n_inst_dev)
        return invalid("null pointer argument");
    if (v->n_gv > 0 && (!splats || !tiles || !values || !inst_first || !entries || !inst_grad))
        return invalid("null pointer argument");
    if (inst_capacity < 0 || inst_capacity > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    PG_CHECK_HIP(launch_render_bwd(v, splats, tiles, values, tile_ranges, tile_order, inst_first, tile_entries, entries,
                                   n_contrib, bg, final_T, dL_dimage, n_inst_dev, inst_capacity, inst_grad, nullptr,
                                   (hipStream_t)stream),
                 "pg_render_bwd");
    return PG_OK;
}

pg_status pg_render_bwd_l1(const pg_views* v, const pg_splat* splats, const pg_tile_set* tiles,
                           const int32_t* values, const int32_t* tile_ranges, const int32_t* tile_order,
                           const int32_t* inst_first, const int64_t* n_inst_dev, int64_t inst_capacity,
                           const int32_t* tile_entries, const uint32_t* entries, const int32_t* n_contrib,
                           const float* bg, const float* final_T, const float* image, const float* target, int64_t n,
                           double* tile_loss, float* inst_grad, void* stream) {
    g_error.clear();
    if (!v || !bg) return invalid("null argument");
    if (!tile_ranges || !tile_entries || !n_contrib || !final_T || !image || !target || !tile_loss || !n_inst_dev)
        return invalid("null pointer argument");
    if (v->n_gv > 0 && (!splats || !tiles || !values || !inst_first || !entries || !inst_grad))
        return invalid("null pointer argument");
    if (inst_capacity < 0 || inst_capacity > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    if (n < 3 * v->n_pixels) return invalid("n must count at least this table's 3 n_pixels floats");
    const BwdL1 l1{image, target, n, tile_loss};
    PG_CHECK_HIP(launch_render_bwd(v, splats, tiles, values, tile_ranges, tile_order, inst_first, tile_entries, entries,
                                   n_contrib, bg, final_T, nullptr, n_inst_dev, inst_capacity, inst_grad, &l1,
                                   (hipStream_t)stream),
                 "pg_render_bwd_l1");
    return PG_OK;
}

pg_status pg_loss_l1_tiles(const double* tile_loss, int64_t n_tiles, int64_t n, float* loss_dev, void* stream) {
    g_error.clear();
    if (!tile_loss || !loss_dev) return invalid("null pointer argument");
    if (n_tiles < 0 || n < 1) return invalid("need n_tiles >= 0 and n >= 1");
    PG_CHECK_HIP(launch_loss_l1_tiles(tile_loss, n_tiles, n, loss_dev, (hipStream_t)stream), "pg_loss_l1_tiles");
    return PG_OK;
}

pg_status pg_project_bwd(const pg_views* v, const float* params, const pg_splat* splats, const pg_bin* bins,
                         const int32_t* inst_first,
                         const int64_t* n_inst_dev, int64_t inst_capacity, const float* inst_grad, const int32_t* gauss_texel, const uint8_t* dynamic_mask, int32_t H,
                         int32_t W, float* grad2d, float* dL_datlas, int32_t accumulate, void* stream) {
    g_error.clear();
    if (!v) return invalid("null argument");
    if (!dL_datlas || !n_inst_dev) return invalid("null pointer argument");
    if (v->n_gv > 0 && (!params || !splats || !bins || !inst_first || !inst_grad || !gauss_texel || !grad2d))
        return invalid("null pointer argument");
    if (H < 1 || W < 1 || (int64_t)H * W < v->n_gauss) return invalid("H * W must hold n_gauss texels");
    if (accumulate != 0 && accumulate != 1) return invalid("accumulate must be 0 or 1");
    if (inst_capacity < 0 || inst_capacity > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    hipStream_t s = (hipStream_t)stream;
    PG_CHECK_HIP(launch_slot_sum(v, bins, inst_first, n_inst_dev, inst_capacity, inst_grad, grad2d, s),
                 "pg_project_bwd (slot sums)");
    PG_CHECK_HIP(launch_project_bwd(v, params, splats, grad2d, gauss_texel, dynamic_mask, H, W, dL_datlas, accumulate,
                                    s),
                 "pg_project_bwd");
    return PG_OK;
}

pg_status pg_backward(const pg_views* v, const float* params, const pg_splat* splats, const pg_bin* bins,
                      const pg_tile_set* tiles, const int32_t* values, const int32_t* tile_ranges,
                      const int32_t* tile_order, const int32_t* inst_first, const int64_t* n_inst_dev,
                      int64_t inst_capacity, const int32_t* tile_entries, const uint32_t* entries,
                      const int32_t* n_contrib, const float* bg, const float* final_T, const float* dL_dimage,
                      float* inst_grad, const int32_t* gauss_texel, const uint8_t* dynamic_mask, int32_t H, int32_t W,
                      float* grad2d, float* dL_datlas, int32_t accumulate, void* stream) {
    g_error.clear();
    if (!v || !bg) return invalid("null argument");
    if (!tile_ranges || !tile_entries || !n_contrib || !final_T || !dL_dimage || !n_inst_dev || !dL_datlas)
        return invalid("null pointer argument");
    if (v->n_gv > 0 && (!params || !splats || !bins || !tiles || !values || !inst_first || !entries || !inst_grad ||
                        !gauss_texel || !grad2d))
        return invalid("null pointer argument");
    if (inst_capacity < 0 || inst_capacity > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    if (H < 1 || W < 1 || (int64_t)H * W < v->n_gauss) return invalid("H * W must hold n_gauss texels");
    if (accumulate != 0 && accumulate != 1) return invalid("accumulate must be 0 or 1");
    hipStream_t s = (hipStream_t)stream;
    PG_CHECK_HIP(launch_render_bwd(v, splats, tiles, values, tile_ranges, tile_order, inst_first, tile_entries, entries,
                                   n_contrib, bg, final_T, dL_dimage, n_inst_dev, inst_capacity, inst_grad, nullptr, s),
                 "pg_backward (compositing adjoint)");
    PG_CHECK_HIP(launch_slot_sum(v, bins, inst_first, n_inst_dev, inst_capacity, inst_grad, grad2d, s),
                 "pg_backward (slot sums)");
    PG_CHECK_HIP(launch_project_bwd(v, params, splats, grad2d, gauss_texel, dynamic_mask, H, W, dL_datlas, accumulate,
                                    s),
                 "pg_backward (projection adjoint)");
    return PG_OK;
}

pg_status pg_status_check(const int32_t* overflow_dev, const int64_t* n_inst_dev, int64_t* needed_capacity,
                          void* stream) {
    g_error.clear();
    if (!overflow_dev || !n_inst_dev) return invalid("null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PG_CHECK_HIP(hipStreamIsCapturing(s, &cs), "pg_status_check (hipStreamIsCapturing)");
    if (cs != hipStreamCaptureStatusNone)
        return invalid("pg_status_check synchronises the stream: call it after a graph replay, not during capture");
    int32_t ovf = 0;
    int64_t need = 0;
    PG_CHECK_HIP(hipMemcpyAsync(&ovf, overflow_dev, sizeof ovf, hipMemcpyDeviceToHost, s), "pg_status_check (copy)");
    PG_CHECK_HIP(hipMemcpyAsync(&need, n_inst_dev, sizeof need, hipMemcpyDeviceToHost, s), "pg_status_check (copy)");
    PG_CHECK_HIP(hipStreamSynchronize(s), "pg_status_check (synchronise)");
    if (needed_capacity) *needed_capacity = need;
    if (ovf & 2) {
        set_error("a radix pass of the sort gave up waiting for an earlier tile's counts; outputs are undefined");
        return PG_ERR_HIP;
    }
    if (ovf) {
        set_error("instance capacity overflow: " + std::to_string(need) + " instances needed");
        return PG_ERR_CAPACITY;
    }
    return PG_OK;
}

pg_status pg_workspace_query(const pg_views* v, int32_t H, int32_t W, int64_t inst_capacity, pg_plan* plan) {
    g_error.clear();
    if (!v || !plan) return invalid("null argument");
    if (H < 1 || W < 1 || (int64_t)H * W < v->n_gauss) return invalid("H * W must hold n_gauss texels");
    if ((int64_t)H * W > INT32_MAX) return invalid("H * W exceeds 2^31 - 1");
    if (inst_capacity < 0 || inst_capacity > INT32_MAX) return invalid("inst_capacity must be in [0, 2^31 - 1]");
    std::memset(plan, 0, sizeof *plan);
    const size_t F = (size_t)v->frames, C = (size_t)v->channels, N = (size_t)v->n_gauss;
    const size_t HW = (size_t)H * W, gv = (size_t)v->n_gv, T = (size_t)v->n_tiles, P = (size_t)v->n_pixels;
    const size_t cap = (size_t)inst_capacity;
    plan->params = F * C * N * sizeof(float);
    plan->gauss_texel = N * sizeof(int32_t);
    plan->texel_gauss = HW * sizeof(int32_t);
    plan->n_gauss = sizeof(int64_t);
    plan->fetch_ws = fetch_ws_bytes(H, W);
    plan->visible = F * N;
    plan->splats = gv * sizeof(pg_splat);
    plan->bins = gv * sizeof(pg_bin);
    plan->tile_sets = gv * sizeof(pg_tile_set);
    plan->keys = cap * sizeof(uint32_t);
    plan->values = cap * sizeof(int32_t);
    plan->tile_ranges = 2 * T * sizeof(int32_t);
    plan->tile_order = T * sizeof(int32_t);
    plan->inst_first = gv * sizeof(int32_t);
    plan->n_inst = 2 * sizeof(int64_t);
    plan->overflow = sizeof(int32_t);
    plan->sort_ws = sort_ws_bytes(v, inst_capacity);
    plan->inst_grad = (size_t)kSlotWords * cap * sizeof(float);
    plan->image = 3 * P * sizeof(float);
    plan->final_T = P * sizeof(float);
    plan->n_contrib = P * sizeof(int32_t);
    plan->tile_entries = T * sizeof(int32_t);
    plan->entries = cap * sizeof(uint32_t);
    plan->dL_dimage = 3 * P * sizeof(float);
    plan->grad2d = 9 * gv * sizeof(float);
    plan->dL_datlas = F * C * HW * sizeof(float);
    const size_t parts[] = {plan->params, plan->gauss_texel, plan->texel_gauss, plan->n_gauss, plan->fetch_ws,
                            plan->visible, plan->splats, plan->bins, plan->tile_sets, plan->keys, plan->values,
                            plan->tile_ranges, plan->tile_order, plan->inst_first, plan->n_inst, plan->overflow,
                            plan->sort_ws, plan->inst_grad, plan->image, plan->final_T, plan->n_contrib,
                            plan->tile_entries, plan->entries, plan->dL_dimage, plan->grad2d, plan->dL_datlas};
    size_t total = 0;
    for (size_t b : parts) total += align256(b);
    plan->total = total;
    return PG_OK;
}

pg_status pg_loss_l1(const float* image, const float* target, int64_t n, float* dL_dimage, double* partial,
                     float* loss_dev, void* stream) {
    g_error.clear();
    if (!image || !target || !dL_dimage || !partial || !loss_dev) return invalid("null pointer argument");
    if (n < 1) return invalid("n must be >= 1");
    PG_CHECK_HIP(launch_loss_l1(image, target, n, dL_dimage, partial, loss_dev, (hipStream_t)stream), "pg_loss_l1");
    return PG_OK;
}

pg_status pg_photo_workspace_size(const pg_views* v, size_t* bytes) {
    g_error.clear();
    if (!v || !bytes) return invalid("null argument");
    *bytes = (size_t)(2 * imax(photo_blocks(v), 1)) * sizeof(double);
    return PG_OK;
}

pg_status pg_loss_photo(const pg_views* v, const float* image, const float* target, float lambda_ssim,
                        float* dL_dimage, float* loss_dev, void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    if (!v) return invalid("views is null");
    if (!loss_dev || !ws) return invalid("null pointer argument");
    if (v->n_pixels > 0 && (!image || !target || !dL_dimage)) return invalid("null pointer argument");
    if (!(lambda_ssim >= 0.0f && lambda_ssim <= 1.0f)) return invalid("lambda_ssim must be in [0, 1]");
    if (ws_bytes < (size_t)(2 * imax(photo_blocks(v), 1)) * sizeof(double)) {
        set_error("photometric-loss workspace too small");
        return PG_ERR_WORKSPACE;
    }
    PG_CHECK_HIP(launch_photo(v, image, target, lambda_ssim, dL_dimage, loss_dev, (double*)ws, (hipStream_t)stream),
                 "pg_loss_photo");
    return PG_OK;
}

pg_status pg_loss_regularisers(const float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                               int32_t channels, const int32_t* gauss_texel, int32_t H, int32_t W,
                               const uint8_t* dyn_gauss, float s_max, float w_scale, float w_opacity,
                               float* dL_datlas, float* reg_loss, double* partial, void* stream) {
    g_error.clear();
    if (!n_gauss_dev || !reg_loss || !partial || !dL_datlas) return invalid("null pointer argument");
    if (n_cap < 0 || (n_cap > 0 && (!params || !gauss_texel))) return invalid("params / gauss_texel null");
    if (frames < 1 || channels < 11 || H < 1 || W < 1) return invalid("bad sizes (need frames >= 1, channels >= 11)");
    if (!std::isfinite(s_max) || !std::isfinite(w_scale) || !std::isfinite(w_opacity)) return invalid("weights must be finite");
    PG_CHECK_HIP(launch_regularisers(params, n_gauss_dev, n_cap, frames, channels, gauss_texel, (int64_t)H * W,
                                     dyn_gauss, s_max, w_scale, w_opacity, dL_datlas, reg_loss, partial,
                                     (hipStream_t)stream),
                 "pg_loss_regularisers");
    return PG_OK;
}

static pg_status uv_prune_check(int64_t n_cap, int32_t frames, int32_t M, int32_t Nv) {
    if (n_cap < 0 || frames < 1 || M < 1 || Nv < 1) return invalid("need n_cap >= 0, frames, M, Nv >= 1");
    if ((int64_t)frames * M * Nv + 1 >= INT32_MAX) return invalid("frames * M * Nv must stay below 2^31");
    if ((int64_t)frames * n_cap >= INT32_MAX) return invalid("frames * n_cap must stay below 2^31");
    return PG_OK;
}

pg_status pg_uv_prune_workspace_size(int64_t n_cap, int32_t frames, int32_t M, int32_t Nv, size_t* bytes) {
    g_error.clear();
    if (!bytes) return invalid("null argument");
    const pg_status st = uv_prune_check(n_cap, frames, M, Nv);
    if (st != PG_OK) return st;
    *bytes = uv_prune_ws_bytes(n_cap, frames, M, Nv);
    return PG_OK;
}

pg_status pg_uv_prune(const float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                      int32_t channels, int32_t M, int32_t Nv, int32_t K, const int32_t* expected_uv, int32_t* uv,
                      int32_t* rank, uint8_t* keep, void* ws, size_t ws_bytes, void* stream) {
    g_error.clear();
    const pg_status st = uv_prune_check(n_cap, frames, M, Nv);
    if (st != PG_OK) return st;
    if (channels < 11 || K < 0) return invalid("need channels >= 11 and K >= 0");
    if (!n_gauss_dev || !ws) return invalid("null pointer argument");
    if (n_cap > 0 && (!params || !uv || !rank || !keep)) return invalid("null pointer argument");
    if (ws_bytes < uv_prune_ws_bytes(n_cap, frames, M, Nv)) {
        set_error("UV pruning workspace too small");
        return PG_ERR_WORKSPACE;
    }
    PG_CHECK_HIP(launch_uv_prune(params, n_gauss_dev, n_cap, frames, channels, M, Nv, K, expected_uv, uv, rank, keep,
                                 ws, (hipStream_t)stream),
                 "pg_uv_prune");
    return PG_OK;
}

pg_status pg_flow_mask(const pg_views* v, const float* params, const uint8_t* flow_masks, uint8_t* tile_motion,
                       uint8_t* dyn_gauss, const int32_t* texel_gauss, int32_t H, int32_t W, uint8_t* dyn_texel,
                       uint64_t* counters, void* stream) {
    g_error.clear();
    if (!v) return invalid("views is null");
    if (v->n_gv > 0 && (!params || !flow_masks || !dyn_gauss || !tile_motion)) return invalid("null pointer argument");
    if (dyn_texel && (!texel_gauss || H < 1 || W < 1)) return invalid("dyn_texel needs texel_gauss and H, W >= 1");
    PG_CHECK_HIP(launch_flow_mask(v, params, flow_masks, tile_motion, dyn_gauss, texel_gauss, dyn_texel ? (int64_t)H * W : 0,
                                  dyn_texel, counters, (hipStream_t)stream),
                 "pg_flow_mask");
    return PG_OK;
}

pg_status pg_atlas_fake_quant(float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                              int32_t channels, const int32_t* bits, float* range, uint16_t* codes, float* partial,
                              void* stream) {
    g_error.clear();
    if (!n_gauss_dev || !bits || !range || !partial) return invalid("null pointer argument");
    if (n_cap < 0 || (n_cap > 0 && !params)) return invalid("params is null with n_cap > 0");
    if (frames < 1 || channels < 1 || channels > kMaxQuantChannels) return invalid("need frames >= 1, 1 <= channels <= 64");
    if ((int64_t)frames * channels > 65535) return invalid("frames * channels must be <= 65535");
    if (n_cap > ((int64_t)1 << 31)) return invalid("n_cap must be <= 2^31");
    for (int c = 0; c < channels; c++)
        if (bits[c] < 0 || bits[c] > 16) return invalid("bits must be in [0, 16]");
    PG_CHECK_HIP(launch_fake_quant(params, n_gauss_dev, n_cap, frames, channels, bits, range, codes, partial,
                                   (hipStream_t)stream),
                 "pg_atlas_fake_quant");
    return PG_OK;
}

pg_status pg_adam_step(float* atlas, const float* grad, float* m, float* v, const uint8_t* visible,
                       const int32_t* texel_gauss, int64_t n_gauss, int32_t frames, int32_t channels, int32_t H,
                       int32_t W, float lr, float beta1, float beta2, float eps, int32_t step, int32_t* step_dev,
                       void* stream) {
    g_error.clear();
    if (!atlas || !grad || !m || !v || !visible || !texel_gauss) return invalid("null pointer argument");
    if (frames < 1 || frames > 65535 || channels < 1 || H < 1 || W < 1 || n_gauss < 0) return invalid("bad sizes");
    if (!step_dev && step < 1) return invalid("step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return invalid("need 0 <= beta < 1 and eps > 0");
    PG_CHECK_HIP(launch_adam(atlas, grad, m, v, visible, texel_gauss, n_gauss, frames, channels, H, W, lr, beta1,
                             beta2, eps, step, step_dev, (hipStream_t)stream),
                 "pg_adam_step");
    return PG_OK;
}

}  // extern "C"
