/*
 * packuv_gs.h -- C ABI of the PackUV-GS differentiable splatting library
 * (MI355X / gfx950).
 *
 * The library renders Gaussians stored in UV-atlas texels (one atlas per
 * frame) into pinhole views and returns the gradient of a loss back to the
 * texels: the "Fitting UV Maps Directly" step of PackUV (arXiv 2602.23040,
 * Sec. 4.2) with the 3DGS tile rasteriser the paper names (Sec. 3,
 * Preliminaries), the EWA projection of Sec. 4.2 / Algorithm 1 and the
 * compositing formula of the supplementary viewer section.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers marked "device" are HIP device pointers owned by the caller;
 *    the library never allocates, frees or retains caller memory.  Pointers
 *    marked "host" are read during the call only.
 *  - `stream` is a hipStream_t (passed as void*).  Every compute call only
 *    enqueues work on it and returns; none synchronises, allocates or issues
 *    memset/memcpy nodes, so a sequence of calls can be captured in a HIP
 *    graph.  The only calls that allocate are pg_views_create (device copy of
 *    the camera table) and pg_views_destroy (frees it).
 *  - Host-detectable problems (null pointers, bad sizes, unsupported tile
 *    shapes, a device that is not gfx950) return an error code before
 *    anything is enqueued; pg_last_error() gives a message (thread-local).
 *  - Device-detected instance-capacity overflow sets *overflow_dev = 1 and
 *    leaves the sorted outputs undefined; *n_inst_dev holds the capacity
 *    that would have sufficed.  NaN inputs propagate; there are no checks on
 *    the hot path.
 *  - Forward and adjoint outputs are bitwise deterministic (fixed reduction
 *    orders, no floating-point atomics).
 *
 * Data layouts
 * ------------
 *  atlas      float [F][C][H][W], C = 11 + 3 (L+1)^2 channels per texel:
 *             x y z | log-scale x y z | quaternion w x y z | logit-opacity |
 *             SH k[j][ch] at channel 11 + 3 j + ch (j = l^2 + l + m).
 *  occupancy  uint8 [H][W]; shared by all F frames.  Occupied texels in
 *             row-major order are the Gaussians of each frame; Gaussian i of
 *             frame f has global id g = f N + i.
 *  params     float [F][C][N]: the occupied texels' raw channels.
 *  views      V cameras; camera v renders frame cams[v].frame.  Per-view
 *             records (pg_splat, pg_bin, 2D gradients) are indexed
 *             gv = v N + i.  Tiles of view v are numbered
 *             tile_base[v] + ty TX_v + tx; pixels pixel_base[v] + y W_v + x.
 *  image      float, view v at offset 3 pixel_base[v], planar [3][H_v][W_v].
 */
#ifndef PACKUV_GS_H
#define PACKUV_GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PG_OK = 0,
    PG_ERR_INVALID_ARG = -1,
    PG_ERR_UNSUPPORTED_DEVICE = -2,
    PG_ERR_CAPACITY = -3,
    PG_ERR_HIP = -4,
    PG_ERR_WORKSPACE = -5
} pg_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward): x_c = R x + t.
 * Pixel (i, j) has centre (i + 0.5, j + 0.5).  Viewer projection of the
 * supplementary viewer section; Jacobian of Algorithm 1. */
typedef struct pg_camera {
    double R[9];            /* world -> camera rotation, row-major */
    double t[3];
    double fx, fy, cx, cy;  /* pixels */
    int32_t width, height;  /* pixels, >= 1 */
    int32_t frame;          /* atlas frame this view renders, 0 <= frame < F */
    int32_t reserved;       /* must be 0 */
} pg_camera;

/* Screen tiling.  tile_w x tile_h must be 256 pixels: 16x16, 8x32 or 32x8
 * (width x height).  lds_batch: Gaussians staged in LDS per step of the
 * compositing loop, one of 64, 128, 256. */
typedef struct pg_tiling {
    int32_t tile_w, tile_h;
    int32_t lds_batch;
    int32_t reserved;       /* must be 0 */
} pg_tiling;

/* Projected Gaussian in one view: what the compositing kernels read. */
typedef struct pg_splat {
    double mean[2];         /* pixel-space mean m (FP64 so tile-local offsets stay exact) */
    float conic[3];         /* (a, b, c) = inverse of Sigma2D: q = a dx^2 + 2 b dx dy + c dy^2 */
    float opacity;          /* sigmoid(logit-opacity) */
    float color[3];         /* max(0, 0.5 + sum_j Y_j(d) k_j), d = unit (mu - camera centre) */
    float depth;            /* fp32(z_c) */
} pg_splat;                 /* 48 bytes */

/* Binning record of a projected Gaussian. */
typedef struct pg_bin {
    int16_t rect[4];        /* x_lo, y_lo, x_hi, y_hi: inclusive tile range */
    uint32_t depth_key;     /* bit pattern of fp32(z_c) (z_c > 0, so it orders like z_c) */
    int32_t n_tiles;        /* kept tiles of rect (pg_project); 0 when culled */
} pg_bin;                   /* 16 bytes */

/* Kept tiles of a (view, Gaussian) record, as pg_project leaves them for the
 * sort's emission and the adjoint's slot lookup (one 16-byte read). */
typedef struct pg_tile_set {
    uint64_t mask;          /* bit (ty - y_lo) w + (tx - x_lo) set for each kept tile of a
                               rectangle of w x h <= 64 tiles; 0: every tile of the rectangle */
    int16_t x_lo, y_lo;     /* rectangle origin, in tiles */
    uint16_t width, height; /* rectangle size in tiles; all fields 0 for culled records */
} pg_tile_set;              /* 16 bytes */

typedef struct pg_views pg_views;   /* opaque: camera table + tiling, resident on the device */

typedef struct pg_views_info {
    int32_t n_views, frames;
    int64_t n_gauss;        /* Gaussians per frame (N) */
    int32_t sh_degree, channels;
    int64_t n_gv;           /* n_views * N */
    int64_t n_tiles;        /* sum over views of TX_v * TY_v */
    int64_t n_pixels;       /* sum over views of W_v * H_v */
    int32_t key_bits;       /* bits of a global tile id (the instance sort key) */
    int32_t sort_passes;    /* radix passes per pg_bin_sort (record sort + instance sort) */
    int32_t tile_w, tile_h, lds_batch, reserved;
} pg_views_info;

/* Selects `device` for the calling thread and checks it is gfx950
 * (PG_ERR_UNSUPPORTED_DEVICE otherwise), then looks up that device's copy of
 * the fixed scratch array that pg_atlas_fetch_noalloc uses. */
pg_status pg_init(int32_t device);

/* Message for the last error of the calling thread ("" if none). */
const char* pg_last_error(void);

/* Builds the device-resident view table for V cameras over `frames` atlases
 * of `n_gauss` Gaussians each (SH degree 0..3).  cams: host [V].  Fails with
 * PG_ERR_INVALID_ARG on bad cameras (fx, fy <= 0, size < 1, frame out of
 * range), unsupported tiling, when frames exceeds 65535 (the projection
 * kernels launch one grid row per frame), when n_gauss exceeds 2^28, or when
 * V * n_gauss or the tile count exceed 2^31 - 1.  Allocates device memory (the only
 * allocating call). */
pg_status pg_views_create(const pg_camera* cams, int32_t n_views, int32_t frames, int64_t n_gauss,
                          int32_t sh_degree, pg_tiling tiling, pg_views** out);
pg_status pg_views_destroy(pg_views* views);
pg_status pg_views_get_info(const pg_views* views, pg_views_info* info);
/* Host arrays of n_views + 1 entries: tile_base[v], pixel_base[v] (last = totals). */
pg_status pg_views_offsets(const pg_views* views, int64_t* tile_base, int64_t* pixel_base);

/* Workspace bytes for pg_atlas_fetch on an H x W atlas. */
pg_status pg_fetch_workspace_size(int32_t H, int32_t W, size_t* bytes);
/* Workspace bytes for pg_bin_sort with room for inst_capacity instances. */
pg_status pg_sort_workspace_size(const pg_views* views, int64_t inst_capacity, size_t* bytes);

/* Byte sizes of every device buffer one fitting step (pg_atlas_fetch ->
 * pg_project -> pg_bin_sort -> pg_render_fwd -> loss -> pg_backward) needs
 * for a view table, an H x W atlas and an instance capacity, besides the
 * atlas itself: the problem statement's "optimise U, render the views,
 * return the gradient" (Sec. 4.2 "Fitting UV Maps Directly") planned ahead.
 * Each field is the size of the buffer of the same name in the calls below;
 * total is their sum with each rounded up to 256 bytes (one allocation that
 * holds them all). */
typedef struct pg_plan {
    size_t params, gauss_texel, texel_gauss, n_gauss, fetch_ws;        /* pg_atlas_fetch */
    size_t visible, splats, bins, tile_sets;                           /* pg_project */
    size_t keys, values, tile_ranges, tile_order, inst_first, n_inst, overflow, sort_ws;  /* pg_bin_sort */
    size_t inst_grad;                                                  /* the adjoint's gradient slots */
    size_t image, final_T, n_contrib, tile_entries, entries;           /* pg_render_fwd */
    size_t dL_dimage;                                                  /* loss cotangent */
    size_t grad2d, dL_datlas;                                          /* pg_backward */
    size_t total;
} pg_plan;
/* Host only: no device work, no synchronisation.  PG_ERR_INVALID_ARG when
 * H W cannot hold n_gauss texels, H W > 2^31 - 1 or inst_capacity is outside
 * [0, 2^31 - 1]. */
pg_status pg_workspace_query(const pg_views* views, int32_t H, int32_t W, int64_t inst_capacity, pg_plan* plan);

/* Host-side status of a step whose instance count the device decides (the
 * capacity-overflow convention above).  Synchronises `stream`, then reads
 * *overflow_dev and *n_inst_dev (from pg_bin_sort).  Returns PG_OK, or
 * PG_ERR_CAPACITY when the last sort overflowed; needed_capacity (host, may
 * be NULL) receives the instance count that suffices either way.  After
 * PG_ERR_CAPACITY the step's outputs are undefined: the caller grows the
 * instance buffers (keys, values, entries, inst_grad, the sort workspace)
 * to at least that count and runs the step again -- in a captured graph,
 * re-captures it, since the graph holds the old buffers.  Returns
 * PG_ERR_INVALID_ARG while `stream` is being captured (it must not
 * synchronise there): call it after the replay. */
pg_status pg_status_check(const int32_t* overflow_dev, const int64_t* n_inst_dev, int64_t* needed_capacity,
                          void* stream);

/* a1 -- Atlas fetch (Sec. 4.2 "Fitting UV Maps Directly"; atlas layout
 * Sec. 4.1).  Compacts occupied texels (row-major rank = Gaussian id) and
 * gathers their raw channels.
 *   atlas       device float [F][C][H][W]
 *   occupancy   device uint8 [H][W]
 *   gauss_texel device int32 [n_cap] out: texel index y W + x of Gaussian i
 *   texel_gauss device int32 [H W]  out: Gaussian id of a texel, -1 if empty
 *   params      device float [F][C][n_cap] out (row stride n_cap)
 *   n_gauss_dev device int64 [1] out: N (ids >= n_cap are not written)
 *   ws          device workspace of pg_fetch_workspace_size bytes */
pg_status pg_atlas_fetch(const float* atlas, const uint8_t* occupancy, int32_t frames, int32_t channels,
                         int32_t H, int32_t W, int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss,
                         float* params, int64_t* n_gauss_dev, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free form of pg_atlas_fetch, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, outputs and results as
 * pg_atlas_fetch (bit-identical), without the workspace: the compaction's
 * block counts and their scan live in a fixed array of
 * PG_FETCH_NOALLOC_SCRATCH_BYTES inside the library, one copy per GPU,
 * which each GPU the library runs on holds until the process ends.  The call
 * allocates and frees nothing.
 *   - H W above PG_FETCH_NOALLOC_MAX_TEXELS (8192 x 8192) returns
 *     PG_ERR_WORKSPACE before anything is enqueued.
 *   - The array's address on a device is looked up by pg_init(device), or
 *     else by the first call on that device; call pg_init before capturing
 *     a graph that holds this call.  The stream must belong to the calling
 *     thread's current device.
 *   - Every call on one GPU shares that GPU's array (it keeps the last
 *     call's contents; nothing in it needs to start at zero): calls that
 *     overlap on one GPU (two streams, two threads) race, and give
 *     undefined results.  Calls in order on one stream are safe. */
#define PG_FETCH_NOALLOC_MAX_TEXELS (1LL << 26)
#define PG_FETCH_NOALLOC_SCRATCH_BYTES (256u * 1024u)
pg_status pg_atlas_fetch_noalloc(const float* atlas, const uint8_t* occupancy, int32_t frames, int32_t channels,
                                 int32_t H, int32_t W, int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss,
                                 float* params, int64_t* n_gauss_dev, void* stream);

/* Low-precision optimisation (LPO) -- the uniform K-bit fake quantiser the
 * renderer consumes instead of the FP32 master texel values (Sec. 4.3 LPO
 * paragraph; supplementary low-precision training section), with the
 * per-channel min/max normalisation of the supplementary video-coding
 * section.  Replaces the fetched values in place by their proxy: for channel
 * c with K = bits[c] in [1, 16], lo / hi = min / max over the fetched
 * Gaussians of every frame, delta = (hi - lo) / (2^K - 1),
 * code = clamp(rint((v - lo) / delta), 0, 2^K - 1), proxy = lo + code delta,
 * each step one FP32 operation rounded to nearest (rint: ties to even);
 * delta = 0 gives code 0.  The paper's widths are 16 bits for the position
 * and 8 for scale, rotation, opacity and colour.  Nothing changes in the
 * adjoint: the straight-through estimator passes the gradient at the proxy
 * to the FP32 master texels as it is (pg_project_bwd's output).
 *   params       device float [F][C][n_cap] in/out (from pg_atlas_fetch)
 *   n_gauss_dev  device int64 [1] (from pg_atlas_fetch); min(N, n_cap) values
 *                per row are used
 *   bits         host int32 [C], C <= 64: 0 leaves a channel unchanged
 *   range        device float [C][2] out: (lo, hi); (0, 0) for channels left
 *                alone or without values
 *   codes        device uint16 [F][C][n_cap] out or NULL: the integer code of
 *                each value (0 in channels left alone); 16-bit codes are what
 *                the storage splits into two 8-bit planes
 *   partial      device float [2 PG_QUANT_BLOCKS C] workspace */
#define PG_QUANT_BLOCKS 256
pg_status pg_atlas_fake_quant(float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                              int32_t channels, const int32_t* bits, float* range, uint16_t* codes, float* partial,
                              void* stream);

/* a2 -- EWA projection (Sec. 4.2 masking equations; Algorithm 1 steps 1-4;
 * viewer projection).  For every view and every Gaussian of its frame:
 * activations s = exp(l_s), unit quaternion, o = sigmoid(l_o); mu_c = R mu + t,
 * cull z_c <= 0.2; Sigma2D = J R Sigma R^T J^T + 0.3 I; cull det <= 1e-7;
 * radius ceil(3 sqrt(lambda_max)); tile rectangle; conic; SH colour.
 * Tile culling by the ellipse: of a rectangle of at most 64 tiles, a tile is
 * kept when the least q over the rectangle of its pixel centres is at most
 * 9.001 (q = 0 when the mean is inside; else the least of the four edge
 * minima, each taken at the edge parabola's clamped vertex); larger
 * rectangles keep every tile.  A record with no kept tile is not listed.  The
 * method lists every tile of the rectangle; the dropped tiles have q > 9 at
 * every pixel centre, so the image and the gradients do not change.
 * Decision quantities are evaluated in FP64 in a fixed order without
 * contraction, from the FP32 texel values.
 *   params     device float [F][C][n_gauss] (row stride n_gauss)
 *   splats     device pg_splat [n_gv] out
 *   bins       device pg_bin [n_gv] out
 *   tiles      device pg_tile_set [n_gv] out: each record's kept tiles
 *   visible    device uint8 [F n_gauss]: set to 1 for Gaussians that survive the z
 *              and det culls in at least one view of this call with a pixel of that
 *              view within r of the mean on both axes (m_x + r >= 0, m_x - r < W,
 *              m_y + r >= 0, m_y - r < H: the rectangle with one-pixel tiles is not
 *              empty).  It does not depend on the tile shape or the tile culling;
 *              never cleared (OR semantics).  The set sparse Adam updates. */
pg_status pg_project(const pg_views* views, const float* params, pg_splat* splats, pg_bin* bins,
                     pg_tile_set* tiles, uint8_t* visible, void* stream);

/* UV-based pruning (Sec. 4.2 "UV-Based Pruning", with the UV projection
 * equation of Sec. 3).  Each fetched Gaussian's position gives its UV pixel
 * on an M x Nv map: u = floor((pi + atan2(y, x)) / (2 pi) M),
 * v = floor(acos(z / rho) / pi Nv) (FP64; theta = pi wraps to u = 0,
 * phi = pi stays in the last row; rho = 0 is invalid).  Valid UV
 * projection: with expected_uv given, a Gaussian that does not map to its
 * entry there is invalid.  Max-K: per frame and pixel, the K valid
 * Gaussians of highest opacity are kept (by the logit; ties by ascending
 * id).  Outputs for the first min(N, n_cap) Gaussians of each frame:
 *   uv           device int32 [F][n_cap] out: v M + u, -1 if invalid
 *   rank         device int32 [F][n_cap] out: rank in the pixel by opacity,
 *                -1 if invalid
 *   keep         device uint8 [F][n_cap] out: 1 for the kept Gaussians
 *   expected_uv  device int32 [F][n_cap] or NULL
 *   ws           device workspace of pg_uv_prune_workspace_size bytes
 * F M Nv and F n_cap must stay below 2^31. */
pg_status pg_uv_prune_workspace_size(int64_t n_cap, int32_t frames, int32_t M, int32_t Nv, size_t* bytes);
pg_status pg_uv_prune(const float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                      int32_t channels, int32_t M, int32_t Nv, int32_t K, const int32_t* expected_uv, int32_t* uv,
                      int32_t* rank, uint8_t* keep, void* ws, size_t ws_bytes, void* stream);

/* Covariance-aware flow masking (Sec. 4.2 "Covariance-Aware Gaussian
 * Masking"; Algorithm 1): the dynamic labels D that gradient freezing uses.
 * For every view and every Gaussian of its frame: the projection of
 * pg_project (same FP64 chain and culls; a culled projection leaves the
 * Gaussian static for that view) and the radius r = ceil(3 sqrt(lambda_max));
 * the Gaussian is dynamic for the view when a pixel whose centre is within r
 * of the mean on both axes, inside the image, has q <= 9 (FP64, at the pixel
 * centre) and a non-zero flow mask.  D is the OR over the views of the
 * Gaussian's frame (the paper's OR across cameras).
 *   params       device float [F][C][n_gauss] (from pg_atlas_fetch)
 *   flow_masks   device uint8 [n_pixels]: view v's [H_v][W_v] mask at its
 *                pixel base; non-zero = motion
 *   tile_motion  device uint8 [n_tiles] workspace: which screen tiles of the
 *                view table hold motion (filled by the call)
 *   dyn_gauss    device uint8 [F][n_gauss] out: D per frame and Gaussian
 *   texel_gauss  device int32 [H W] (from pg_atlas_fetch); read only with
 *   dyn_texel    device uint8 [H W] out or NULL: 1 where the texel's Gaussian
 *                is dynamic in some frame (the mask pg_project_bwd takes)
 *   counters     device uint64 [1] or NULL: += pixel centres tested */
pg_status pg_flow_mask(const pg_views* views, const float* params, const uint8_t* flow_masks, uint8_t* tile_motion,
                       uint8_t* dyn_gauss, const int32_t* texel_gauss, int32_t H, int32_t W, uint8_t* dyn_texel,
                       uint64_t* counters, void* stream);

/* a3 -- Tile binning and depth sort (tile rasteriser, Sec. 3; per-camera
 * depth sort, viewer section).  Lists every surviving (view, Gaussian) once
 * per kept tile of its rectangle and orders each tile's list front to back by
 * fp32(z_c), equal depths by ascending Gaussian id.  Implementation: the
 * surviving records, taken in (view, id) order, are stably radix-sorted by
 * depth; instances are emitted in that order and stably radix-sorted by
 * global tile id (a tile belongs to one view, so its list ends up ordered by
 * (depth, id)).
 *   bins, tiles    from pg_project
 *   keys           device uint32 [inst_capacity] out: global tile of each
 *                  sorted instance (ascending)
 *   values         device int32 [inst_capacity] out: gv of each sorted instance
 *   tile_ranges    device int32 [n_tiles][2] out: [start, end) per tile
 *   tile_order     device int32 [n_tiles] out, or NULL: a dispatch order for
 *                  the compositing calls, every tile once, longest lists
 *                  first (64 classes of list length, four per octave; the
 *                  order inside a class is not deterministic).  It only
 *                  schedules work: results do not depend on it
 *   inst_first     device int32 [n_gv] out: the number of instances of all
 *                  records before gv in (view, id) order.  The adjoint keeps
 *                  one gradient slot per instance, record by record in that
 *                  order, the record's kept tiles in rectangle row-major order.
 *   n_inst_dev     device int64 [2] in/out: [0] out: number of instances;
 *                  [1] the sort generation, advanced by one (skipping 0) on
 *                  every call.  The adjoint tags the gradient slots it writes
 *                  with it, and slots with another tag read as zero, so the
 *                  slots are never cleared: allocate n_inst_dev and the
 *                  slots (pg_render_bwd's inst_grad) zero-filled once.
 *   overflow_dev   device int32 [1] out: bit 0 set if n_inst > inst_capacity;
 *                  bit 1 set if a radix pass gave up waiting on an earlier
 *                  tile's counts (never in a working run; pg_status_check
 *                  then returns PG_ERR_HIP); 0 otherwise
 *   ws             device workspace of pg_sort_workspace_size bytes */
pg_status pg_bin_sort(const pg_views* views, const pg_bin* bins, const pg_tile_set* tiles, int64_t inst_capacity,
                      uint32_t* keys,
                      int32_t* values, int32_t* tile_ranges, int32_t* tile_order, int32_t* inst_first,
                      int64_t* n_inst_dev, int32_t* overflow_dev, void* ws, size_t ws_bytes,
                      void* stream);

/* a4 -- Front-to-back compositing (supplementary viewer section:
 * C = sum_i T_i alpha_i c_i, T_i = prod_{j<i} (1 - alpha_j); footprint
 * d^2 <= 9 of Sec. 4.2).  Per pixel: skip q > 9; alpha = min(0.99, o e^{-q/2});
 * skip alpha < 1/255; stop before T (1 - alpha) < 1e-4.  Writes C + T bg.
 * Also records, for the adjoint, which pixels composited which Gaussian.
 *   tile_ranges  from pg_bin_sort
 *   tile_order   device int32 [n_tiles] from pg_bin_sort, or NULL: the order
 *                in which tiles are dispatched (NULL: neighbouring tiles
 *                together); a tile index outside [0, n_tiles) is skipped
 *   bg           host float[3]
 *   image        device float [3 n_pixels] out (per view planar [3][H][W])
 *   final_T      device float [n_pixels] out
 *   n_contrib    device int32 [n_pixels] out: list positions the pixel
 *                reached: the 0-based position of the Gaussian at which it
 *                stopped (T would have dropped below 1e-4), else the length
 *                of its tile's list
 *   tile_entries device int32 [n_tiles] out: number of entries of each tile
 *   entries      device uint32 [inst_capacity] out: for tile t, words
 *                [start_t, start_t + tile_entries[t]) describe, in ascending
 *                list order, the Gaussians that composited at least one
 *                pixel of the tile: (0-based list position << 4) | bit b set
 *                when a pixel of the tile's 8x8 block b (row-major) took it.
 *                A tile's list never exceeds n_gauss <= 2^28, so the
 *                position fits.
 *   counters     device uint64 [2] or NULL: += {pairs evaluated, pairs composited} */
pg_status pg_render_fwd(const pg_views* views, const pg_splat* splats, const int32_t* values,
                        const int32_t* tile_ranges, const int32_t* tile_order, const float* bg, float* image,
                        float* final_T,
                        int32_t* n_contrib, int32_t* tile_entries, uint32_t* entries, uint64_t* counters,
                        void* stream);

/* a5, first half -- Adjoint of the compositing (a4) per screen tile.  Walks
 * each tile's entries back to front with the forward's decisions,
 * recomputing per-pixel transmittance from final_T instead of storing it,
 * and writes each (Gaussian, tile) instance's sums over the tile's pixels to
 * that instance's own slot (no atomics): with dq' = alpha dL/dalpha (so
 * dL/dq = -dq'/2) and (dx, dy) = pixel - mean, the nine floats are
 * sum dq' dx, sum dq' dy, sum dq' dx^2, sum dq' dx dy, sum dq' dy^2, sum dq'
 * and dL/d(r, g, b).  The mean and conic gradients are linear in the first
 * five and dL/dopacity is sum dq' / opacity; pg_project_bwd forms them per
 * record.  A slot is 10 words: the
 * nine sums, then the sort generation (n_inst_dev[1], as uint32 bits) that
 * marks it as written by this step.  Slots of instances that composited
 * nothing are not written: they keep an older tag (or the zero of a
 * zero-filled buffer) and pg_project_bwd counts them as zero.
 *   tile_ranges, tile_order   as for pg_render_fwd
 *   tiles, inst_first, n_inst_dev   from pg_project / pg_bin_sort; after an
 *                overflowed sort (n_inst > inst_capacity) no slot is written
 *   tile_entries, entries, n_contrib, final_T   from pg_render_fwd
 *   dL_dimage    device float [3 n_pixels]
 *   inst_capacity the capacity given to pg_bin_sort
 *   inst_grad    device float [inst_capacity][10] in/out, zero-filled when
 *                allocated (never cleared afterwards), slot inst_first[gv] + k
 *                for the k-th kept tile (row-major) of record gv's rectangle */
pg_status pg_render_bwd(const pg_views* views, const pg_splat* splats, const pg_tile_set* tiles,
                        const int32_t* values, const int32_t* tile_ranges, const int32_t* tile_order,
                        const int32_t* inst_first, const int64_t* n_inst_dev,
                        int64_t inst_capacity, const int32_t* tile_entries, const uint32_t* entries,
                        const int32_t* n_contrib, const float* bg, const float* final_T, const float* dL_dimage,
                        float* inst_grad, void* stream);

/* a4' and a5 first half together, for the L1 objective of Sec. 4.2
 * "Objective" (lambda_ssim = 0): pg_render_bwd with its cotangent formed per
 * pixel from image and target as sign(image - target) / n, the expression of
 * pg_loss_l1 (so the slots equal those of pg_loss_l1 + pg_render_bwd bit for
 * bit), and each tile's sum of |image - target| (FP64, fixed order) written
 * to tile_loss[tile]; pg_loss_l1_tiles then forms the loss value.  This
 * spares the cotangent's write and read and the L1 pass over the images.
 *   image, target  device float [3 n_pixels] (per view planar [3][H][W])
 *   n              the number of image floats in the whole objective (3
 *                  n_pixels of the table, or more when several tables share
 *                  one loss); the cotangent is 1 / n per float
 *   tile_loss      device double [n_tiles] out (every tile written)
 * The other arguments are those of pg_render_bwd. */
pg_status pg_render_bwd_l1(const pg_views* views, const pg_splat* splats, const pg_tile_set* tiles,
                           const int32_t* values, const int32_t* tile_ranges, const int32_t* tile_order,
                           const int32_t* inst_first, const int64_t* n_inst_dev, int64_t inst_capacity,
                           const int32_t* tile_entries, const uint32_t* entries, const int32_t* n_contrib,
                           const float* bg, const float* final_T, const float* image, const float* target, int64_t n,
                           double* tile_loss, float* inst_grad, void* stream);

/* L = sum(tile_loss[0 .. n_tiles)) / n (FP64, fixed order) into loss_dev
 * (device float [1]): the L1 loss value after pg_render_bwd_l1 (one call
 * for tables whose tile sums lie side by side in tile_loss). */
pg_status pg_loss_l1_tiles(const double* tile_loss, int64_t n_tiles, int64_t n, float* loss_dev, void* stream);

/* a5, second half -- Adjoint of the projection (a2) and the fetch (a1)
 * back to the texels, with gradient freezing grad <- D_i grad (Sec. 4.2
 * "Gradient Freezing").  Adds each record's instance slots in rectangle
 * order (a fixed order, so the result is bitwise deterministic), then
 * applies the chain rule through the EWA projection, the activations and
 * the SH colour of every view of the Gaussian's frame.
 *   splats       from pg_project: the SH adjoint takes a colour channel's clamp
 *                decision (colour = max(0, 0.5 + sum Y k)) from the forward's
 *                stored colour where its own FP32 sum lies within 1e-3 of 0
 *   bins, inst_first, n_inst_dev   from pg_project / pg_bin_sort;
 *                after an overflowed sort the texel gradient is zero
 *   inst_grad    device float [inst_capacity][10] from pg_render_bwd; a slot
 *                counts only when its tag is the current sort generation
 *   gauss_texel  device int32 [n_gauss] (from pg_atlas_fetch)
 *   dynamic_mask device uint8 [H][W] or NULL (NULL: every Gaussian dynamic)
 *   grad2d       device float [9][n_gv] out: per (view, Gaussian) dL/d(m_x,
 *                m_y, a, b, c, opacity, r, g, b) (mean and conic formed from
 *                the summed moments with the FP64 conic); 0 for culled records
 *   dL_datlas    device float [F][C][H][W] out; written (accumulate = 0: every
 *                texel, unoccupied = 0) or added to (accumulate = 1: occupied
 *                texels only). */
pg_status pg_project_bwd(const pg_views* views, const float* params, const pg_splat* splats, const pg_bin* bins,
                         const int32_t* inst_first,
                         const int64_t* n_inst_dev, int64_t inst_capacity, const float* inst_grad, const int32_t* gauss_texel, const uint8_t* dynamic_mask, int32_t H,
                         int32_t W, float* grad2d, float* dL_datlas, int32_t accumulate, void* stream);

/* a5 -- The whole adjoint: dL/dimage in, dL/datlas out, with gradient
 * freezing (Sec. 4.2 "Gradient Freezing"; the problem statement's "return
 * the gradient to U").  Enqueues pg_render_bwd and then pg_project_bwd with
 * the arguments of the same names, so its results are theirs bit for bit;
 * the two halves stay separate entry points for callers that keep the
 * per-instance or per-record gradients.  Argument checks are those of both
 * calls, made before anything is enqueued. */
pg_status pg_backward(const pg_views* views, const float* params, const pg_splat* splats, const pg_bin* bins,
                      const pg_tile_set* tiles, const int32_t* values, const int32_t* tile_ranges,
                      const int32_t* tile_order, const int32_t* inst_first, const int64_t* n_inst_dev,
                      int64_t inst_capacity, const int32_t* tile_entries, const uint32_t* entries,
                      const int32_t* n_contrib, const float* bg, const float* final_T, const float* dL_dimage,
                      float* inst_grad, const int32_t* gauss_texel, const uint8_t* dynamic_mask, int32_t H, int32_t W,
                      float* grad2d, float* dL_datlas, int32_t accumulate, void* stream);

/* a4' -- L1 photometric term of Sec. 4.2 "Objective" (lambda_ssim = 0):
 * L = mean |image - target|, dL/dimage = sign(image - target) / n (sign 0 = 0).
 *   partial   device double [1024] workspace
 *   loss_dev  device float [1] out */
pg_status pg_loss_l1(const float* image, const float* target, int64_t n, float* dL_dimage, double* partial,
                     float* loss_dev, void* stream);

/* Full photometric term of Sec. 4.2 "Objective":
 * L = (1 - lambda_ssim) mean |image - target| + lambda_ssim (1 - mean SSIM),
 * means over every view, pixel and channel, and dL/dimage.  SSIM per channel
 * plane of each view: 11 x 11 Gaussian window (sigma 1.5, weights summing to
 * 1), zero padding outside the view, C1 = 0.01^2, C2 = 0.03^2 (data range 1);
 * its image gradient is the window correlation of its partials with respect
 * to the window sums.  The paper does not give lambda_ssim (0 gives the L1
 * term of pg_loss_l1; 3DGS uses 0.2).  FP32 arithmetic, FP64 sums.
 *   image, target  device float [3 n_pixels] (per view planar [3][H][W])
 *   dL_dimage      device float [3 n_pixels] out
 *   loss_dev       device float [1] out
 *   ws             device workspace of pg_photo_workspace_size bytes */
pg_status pg_photo_workspace_size(const pg_views* views, size_t* bytes);
pg_status pg_loss_photo(const pg_views* views, const float* image, const float* target, float lambda_ssim,
                        float* dL_dimage, float* loss_dev, void* ws, size_t ws_bytes, void* stream);

/* Scale and opacity regularisers of Sec. 4.2 "Objective", over the fetched
 * Gaussians of every frame (or only the dynamic ones):
 *   L_scale = mean max(0, max_k s_k - s_max)^2,  L_opacity = mean o (1 - o),
 * s = exp(l_s), o = sigmoid(l_o), FP64 from the FP32 texel values (the
 * paper's weights are 1e-4 each; s_max is not given).  Adds
 * w_scale dL_scale + w_opacity dL_opacity to the texel gradient (the
 * largest scale's log-scale channel and the logit-opacity channel).
 *   params       device float [F][C][n_cap] (from pg_atlas_fetch)
 *   n_gauss_dev  device int64 [1]; min(N, n_cap) Gaussians per frame
 *   gauss_texel  device int32 [n_cap] (from pg_atlas_fetch)
 *   dyn_gauss    device uint8 [F][n_cap] or NULL (NULL: every Gaussian)
 *   dL_datlas    device float [F][C][H][W], added to
 *   reg_loss     device float [2] out: L_scale, L_opacity
 *   partial      device double [3 PG_REG_BLOCKS + 1] workspace */
#define PG_REG_BLOCKS 256
pg_status pg_loss_regularisers(const float* params, const int64_t* n_gauss_dev, int64_t n_cap, int32_t frames,
                               int32_t channels, const int32_t* gauss_texel, int32_t H, int32_t W,
                               const uint8_t* dyn_gauss, float s_max, float w_scale, float w_opacity,
                               float* dL_datlas, float* reg_loss, double* partial, void* stream);

/* a6 -- Sparse Adam on the FP32 atlas (Sec. 4.3, LPO paragraph: FP32 master
 * weights, Sparse Adam).  Textbook Adam with bias correction at `step` >= 1,
 * applied to channels of texels whose Gaussian is visible (visible[f N + i]);
 * other texels and their moments are left untouched.
 *   atlas, m, v  device float [F][C][H][W] in/out;  grad same layout (F <= 65535)
 *   step         the step number (>= 1) for bias correction, or ignored when
 *   step_dev     (device int32 [1], may be NULL) is given: the call then adds
 *                1 to *step_dev on the device and uses the new value, so the
 *                replays of a captured step count their steps */
pg_status pg_adam_step(float* atlas, const float* grad, float* m, float* v, const uint8_t* visible,
                       const int32_t* texel_gauss, int64_t n_gauss, int32_t frames, int32_t channels, int32_t H,
                       int32_t W, float lr, float beta1, float beta2, float eps, int32_t step, int32_t* step_dev,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PACKUV_GS_H */
