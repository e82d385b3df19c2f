// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "packuv_gs.h"

namespace pg {

constexpr int kMaxViews = 1 << 16;
constexpr int kScanBlocks = 1024;    // fixed grid of the device-length scans
constexpr int kSortThreads = 256;    // radix sort work-group
constexpr int kSortItems = 16;       // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;
// Words of one per-instance gradient slot: nine sums and the generation tag
// (the sort generation the adjoint wrote it in; other slots read as zero).
constexpr int kSlotWords = 10;

// Per-view table resident on the device.
struct ViewDev {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double cw[3];          // camera centre in world coordinates, -R^T t
    float Rf[9], tf[3], fxf, fyf, cwf[3];   // FP32 copies for the adjoint
    int32_t W, H, TX, TY;
    int32_t frame, pad;
    int64_t tile_base, pix_base;
};

}  // namespace pg

struct pg_views {
    int32_t n_views, frames, sh_degree, channels;
    int64_t n_gauss;
    pg_tiling tiling;
    int64_t n_gv, n_tiles, n_pixels;
    int32_t key_bits, sort_passes;
    int32_t device;
    pg::ViewDev* d_views;      // [n_views]
    int32_t* d_frame_views;    // [frames + 1] offsets into d_view_order
    int32_t* d_view_order;     // [n_views] view indices grouped by frame
    int64_t n_ssim_blocks;     // 32 x 32 pixel blocks of all views (photometric loss)
    int64_t* d_ssim_base;      // [n_views] first block of each view
    int64_t* h_tile_base;      // [n_views + 1]
    int64_t* h_pix_base;       // [n_views + 1]
};

namespace pg {

// thread-local error message
void set_error(const std::string& msg);
pg_status hip_fail(hipError_t e, const char* what);

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ inline int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- launchers implemented in the kernel translation units (all enqueue only)

// scan.hip
hipError_t fill_u32(void* p, uint32_t value, int64_t n_words, hipStream_t s);
// exclusive scan of n (device-read: *n_dev * n_mul, or n_host when n_dev == null) int64 values
hipError_t scan_i64(const int64_t* in, int64_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                    int64_t* total_out, int64_t* block_tmp, hipStream_t s);
hipError_t scan_i32_as_i64(const int32_t* in, int64_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                           int64_t* total_out, int64_t* block_tmp, hipStream_t s);
hipError_t scan_i32(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                    int64_t* total_out, int64_t* block_tmp, hipStream_t s);
constexpr int64_t kScanTmpWords = kScanBlocks + 1;   // int64 scratch words a scan needs

// fetch.hip
size_t fetch_ws_bytes(int32_t H, int32_t W);
hipError_t launch_fetch(const float* atlas, const uint8_t* occ, int32_t F, int32_t C, int32_t H, int32_t W,
                        int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss, float* params,
                        int64_t* n_gauss_dev, void* ws, hipStream_t s);

// loss.hip (photometric objective)
int64_t photo_blocks(const pg_views* v);
hipError_t launch_photo(const pg_views* v, const float* image, const float* target, float lambda, float* dimg,
                        float* loss, double* partial, hipStream_t s);
hipError_t launch_regularisers(const float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C,
                               const int32_t* gauss_texel, int64_t HW, const uint8_t* dyn, double s_max,
                               double w_scale, double w_opacity, float* gatlas, float* loss, double* partial,
                               hipStream_t s);

// uvprune.hip
size_t uv_prune_ws_bytes(int64_t n_cap, int32_t F, int32_t M, int32_t Nv);
hipError_t launch_uv_prune(const float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C, int32_t M,
                           int32_t Nv, int32_t K, const int32_t* expected, int32_t* uv, int32_t* rank, uint8_t* keep,
                           void* ws, hipStream_t s);

// quant.hip
constexpr int kMaxQuantChannels = 64;       // channels a fake-quantiser call may hold
constexpr int kQuantBlocks = PG_QUANT_BLOCKS;
hipError_t launch_fake_quant(float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C,
                             const int32_t* bits, float* range, uint16_t* codes, float* partial, hipStream_t s);

// project.hip
hipError_t launch_project(const pg_views* v, const float* params, pg_splat* splats, pg_bin* bins,
                          pg_tile_set* tiles, uint8_t* visible, hipStream_t s);
hipError_t launch_flow_mask(const pg_views* v, const float* params, const uint8_t* masks, uint8_t* tile_motion,
                            uint8_t* dyn_gauss, const int32_t* texel_gauss, int64_t HW, uint8_t* dyn_texel,
                            uint64_t* counters, hipStream_t s);
// per-record sums of the instance slots -> grad2d
hipError_t launch_slot_sum(const pg_views* v, const pg_bin* bins, const int32_t* inst_first,
                           const int64_t* n_inst_dev, int64_t cap, const float* inst_grad, float* grad2d,
                           hipStream_t s);
hipError_t launch_project_bwd(const pg_views* v, const float* params, const pg_splat* splats, float* grad2d,
                              const int32_t* gauss_texel, const uint8_t* dyn, int32_t H, int32_t W,
                              float* dL_datlas, int32_t accumulate, hipStream_t s);

// binsort.hip
size_t sort_ws_bytes(const pg_views* v, int64_t cap);
hipError_t launch_bin_sort(const pg_views* v, const pg_bin* bins, const pg_tile_set* tiles, int64_t cap,
                           uint32_t* keys, int32_t* values,
                           int32_t* ranges, int32_t* tile_order, int32_t* inst_first, int64_t* n_inst_dev,
                           int32_t* overflow_dev, void* ws, hipStream_t s);

// stable sort of (uint32 key, int32 value) pairs (binsort.hip)
size_t sort_pairs_ws_bytes(int64_t cap, int bits);
hipError_t sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, const int64_t* n_dev,
                      int64_t cap, int bits, void* ws, uint32_t** out_keys, int32_t** out_vals, hipStream_t s);

// render.hip
hipError_t launch_render_fwd(const pg_views* v, const pg_splat* splats, const int32_t* values,
                             const int32_t* ranges, const int32_t* order, const float bg[3], float* image,
                             float* final_T, int32_t* n_contrib, int32_t* tile_entries, uint32_t* entries,
                             uint64_t* counters, hipStream_t s);
// The L1 term formed inside the compositing adjoint: its cotangent from image
// and target (n floats in the whole objective), and the tiles' sums of
// |image - target| in tile_loss.
struct BwdL1 {
    const float* image;
    const float* target;
    int64_t n;
    double* tile_loss;
};
// dL_dimage is read when l1 is null; otherwise the cotangent is the L1 term's.
hipError_t launch_render_bwd(const pg_views* v, const pg_splat* splats, const pg_tile_set* tiles, const int32_t* values,
                             const int32_t* ranges, const int32_t* order, const int32_t* inst_first,
                             const int32_t* tile_entries, const uint32_t* entries, const int32_t* n_contrib,
                             const float bg[3], const float* final_T, const float* dL_dimage,
                             const int64_t* n_inst_dev, int64_t cap, float* inst_grad, const BwdL1* l1,
                             hipStream_t s);
hipError_t fill_u32_dev(void* p, uint32_t value, const int64_t* n_dev, int64_t n_max, int64_t mul, hipStream_t s);

// optim.hip
hipError_t launch_loss_l1(const float* img, const float* tgt, int64_t n, float* g, double* partial, float* loss,
                          hipStream_t s);
hipError_t launch_loss_l1_tiles(const double* tile_loss, int64_t n_tiles, int64_t n, float* loss, hipStream_t s);
hipError_t launch_adam(float* atlas, const float* grad, float* m, float* v, const uint8_t* visible,
                       const int32_t* texel_gauss, int64_t n_gauss, int32_t F, int32_t C, int32_t H, int32_t W,
                       float lr, float b1, float b2, float eps, int32_t step, int32_t* step_dev, hipStream_t s);

// ---- device helpers

// Fourth word of a raw buffer resource on gfx9-family chips: 32-bit data
// format, no swizzle, no index stride.  Raw (untyped) buffer accesses bound
// every lane's offset by the resource's byte count; stores past it are
// dropped and loads return 0.
constexpr int kBufWord3 = 0x00020000;

// Kept-tile sets (pg_tile_set, from the projection): bit (ty - y_lo) w +
// (tx - x_lo) of a record's mask is set when that tile of its rectangle is
// kept; a zero mask means every tile is kept.  The record's instances and
// gradient slots follow its kept tiles in rectangle row-major order.

__device__ __forceinline__ int32_t kept_count(const uint4& ts) {
    const uint64_t mask = (uint64_t)ts.x | ((uint64_t)ts.y << 32);
    return mask ? (int32_t)__popcll(mask) : (int32_t)(ts.w & 0xffffu) * (int32_t)(ts.w >> 16);
}

// Index among the kept tiles of the tile at rectangle bit `bit`.
__device__ __forceinline__ int32_t kept_rank(uint64_t mask, int32_t bit) {
    return mask ? (int32_t)__popcll(mask & (((uint64_t)1 << bit) - 1)) : bit;
}

// Cross-lane data-parallel-primitive move of a float: lanes of rows disabled
// by ROW_MASK read 0 (control codes: quad_perm 0x00-0xFF, row_ror:n 0x120+n,
// row_mirror 0x140, row_half_mirror 0x141, row_bcast:15 0x142, row_bcast:31 0x143).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ int find_view_by_tile(const ViewDev* views, int nv, int64_t tile) {
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace pg
