// a4 -- front-to-back compositing per screen tile, and (a5, first half) its
// adjoint per pixel.
//
// Compositing follows C = sum_i T_i alpha_i c_i with T_i = prod_{j<i}
// (1 - alpha_j) (supplementary, viewer section), restricted to the 3-sigma
// ellipse q = d^2 <= 9 of Sec. 4.2; alpha = min(0.99, o e^{-q/2}), Gaussians
// with alpha < 1/255 are skipped, and a pixel stops before the Gaussian that
// would bring T below 1e-4.
//
// Launch shape: one 256-lane work-group (four wave64s) per (view, tile), one
// pixel per lane.  The tile's list is staged through LDS in batches of
// BATCH Gaussians; every lane of the group reads each staged Gaussian as an
// LDS broadcast, so the per-instance HBM record (48 bytes) is reused by up to
// 256 pixels and the loop is bound by FP32 VALU work, not HBM.  A group stops
// loading batches once every lane has terminated (__syncthreads_count).
// Work-groups are assigned to tiles so that consecutive tiles run on the same
// XCD (the dispatcher deals groups round-robin over the 8 XCDs), which keeps
// the records that neighbouring tiles share in one L2.
//
// Pixel offsets are formed in FP32 coordinates local to the 32x32 pixel block
// holding the tile (every supported tile shape nests in such a block), from
// the FP64 pixel-space mean: q keeps full FP32 precision at 1080p, and a
// pixel sees bit-identical inputs whatever the tile shape.
//
// The adjoint walks each pixel's composited Gaussians back to front,
// recovering the transmittance in front of Gaussian k as T_k = T_{k+1} /
// (1 - alpha_k) from the stored final T (no per-step storage).  Per-Gaussian
// sums over the tile's pixels are reduced across the wave (skipped when no
// lane contributes), then across the four waves with LDS float atomics, then
// added to the (view, Gaussian) gradient with one global float atomic per
// value and tile.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr float kQMax = 9.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;

// The one definition of q and alpha used by both the forward and the adjoint,
// with explicit fused multiply-adds so both kernels take bit-identical
// decisions (the library is compiled with -ffp-contract=off).
struct Eval {
    float q, e, raw, alpha;
};

__device__ __forceinline__ float quad(float dx, float dy, float a, float b2, float c) {
    const float u = fmaf(b2, dy, a * dx);      // a dx + 2 b dy
    return fmaf(u, dx, (c * dy) * dy);         // dx (a dx + 2 b dy) + c dy^2
}

__device__ __forceinline__ Eval evaluate(float q, float o) {
    Eval r;
    r.q = q;
    r.e = __expf(-0.5f * q);
    r.raw = o * r.e;
    r.alpha = r.raw < kAlphaMax ? r.raw : kAlphaMax;
    return r;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t i, int64_t n) {
    const int64_t per = n >> 3, rem = n & 7;
    const int64_t x = i & 7, j = i >> 3;
    return x * per + imin(x, rem) + j;
}

struct TileCtx {
    int64_t tile;
    int32_t v, W, H, px, py;
    double ox, oy;
    int64_t pix;
    bool inside;
};

template <int TW, int TH>
__device__ __forceinline__ TileCtx tile_ctx(const ViewDev* views, int nv, int64_t n_tiles) {
    TileCtx c;
    c.tile = xcd_remap(blockIdx.x, n_tiles);
    c.v = find_view_by_tile(views, nv, c.tile);
    const ViewDev& V = views[c.v];
    const int64_t lt = c.tile - V.tile_base;
    const int32_t tx = (int32_t)(lt % V.TX), ty = (int32_t)(lt / V.TX);
    const int32_t lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    c.W = V.W;
    c.H = V.H;
    c.px = tx * TW + lx;
    c.py = ty * TH + ly;
    c.ox = (double)((tx * TW) & ~31);
    c.oy = (double)((ty * TH) & ~31);
    c.inside = c.px < c.W && c.py < c.H;
    c.pix = V.pix_base + (int64_t)c.py * c.W + c.px;
    return c;
}

// Stage Gaussian `gv` into LDS slot `k` in tile-local coordinates.
__device__ __forceinline__ void stage(const pg_splat* __restrict__ splats, int32_t gv, double ox, double oy,
                                      float4* s_geo, float4* s_col, float* s_blu, int k) {
    const float4* sp = reinterpret_cast<const float4*>(splats + gv);
    const float4 a = sp[0], b = sp[1], c = sp[2];
    double2 m;
    *reinterpret_cast<float4*>(&m) = a;
    s_geo[k] = make_float4((float)(m.x - ox), (float)(m.y - oy), b.x, 2.0f * b.y);
    s_col[k] = make_float4(b.z, b.w, c.x, c.y);   // conic c, opacity, red, green
    s_blu[k] = c.z;
}

template <int TW, int TH, int BATCH, bool STATS>
__global__ __launch_bounds__(256) void k_render_fwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                    const pg_splat* __restrict__ splats,
                                                    const int32_t* __restrict__ values,
                                                    const int2* __restrict__ ranges, float bg0, float bg1,
                                                    float bg2, float* __restrict__ image,
                                                    float* __restrict__ final_T, int32_t* __restrict__ n_contrib,
                                                    unsigned long long* __restrict__ counters) {
    __shared__ float4 s_geo[BATCH];
    __shared__ float4 s_col[BATCH];
    __shared__ float s_blu[BATCH];
    const TileCtx c = tile_ctx<TW, TH>(views, nv, n_tiles);
    const int2 rg = ranges[c.tile];
    const float fx = (float)(c.px - (int32_t)c.ox) + 0.5f, fy = (float)(c.py - (int32_t)c.oy) + 0.5f;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t n = 0;
    bool done = !c.inside;
    uint32_t n_eval = 0, n_comp = 0;
    for (int32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
        if (__syncthreads_count(!done) == 0) break;
        const int32_t j = b0 + (int32_t)threadIdx.x;
        if (threadIdx.x < BATCH && j < rg.y) stage(splats, values[j], c.ox, c.oy, s_geo, s_col, s_blu, threadIdx.x);
        __syncthreads();
        const int32_t cnt = min(BATCH, rg.y - b0);
        for (int32_t k = 0; k < cnt; k++) {
            const float4 g = s_geo[k];
            const float dx = fx - g.x, dy = fy - g.y;
            const float4 cc = s_col[k];
            const float q = quad(dx, dy, g.z, g.w, cc.x);
            if (STATS) n_eval += done ? 0u : 1u;
            bool in = !done && q <= kQMax;
            if (!__any(in)) continue;                 // wave-uniform: nobody inside the ellipse
            const Eval ev = evaluate(q, cc.y);
            in = in && ev.alpha >= kAlphaMin;
            const float Tn = T * (1.0f - ev.alpha);
            const bool stop = in && Tn < kTMin;
            const bool take = in && !stop;
            done = done || stop;
            const float w = take ? T * ev.alpha : 0.0f;
            C0 = fmaf(w, cc.z, C0);
            C1 = fmaf(w, cc.w, C1);
            C2 = fmaf(w, s_blu[k], C2);
            T = take ? Tn : T;
            n = take ? b0 - rg.x + k + 1 : n;
            if (STATS) n_comp += take ? 1u : 0u;
            if (!__any(!done)) break;                 // every pixel of the wave has terminated
        }
    }
    if (c.inside) {
        const int64_t HW = (int64_t)c.W * c.H;
        const int64_t vb = c.pix - ((int64_t)c.py * c.W + c.px);   // pixel base of the view
        float* img = image + 3 * vb + (int64_t)c.py * c.W + c.px;
        img[0] = fmaf(T, bg0, C0);
        img[HW] = fmaf(T, bg1, C1);
        img[2 * HW] = fmaf(T, bg2, C2);
        final_T[c.pix] = T;
        n_contrib[c.pix] = n;
    }
    if (STATS) {
        unsigned long long e = n_eval, p = n_comp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            p += __shfl_xor(p, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&counters[0], e);
            atomicAdd(&counters[1], p);
        }
    }
}

// Cross-lane data-parallel-primitive move: lanes of disabled rows read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes of a wave with DPP moves only (no LDS traffic):
// butterflies inside quads, half-row and row mirrors give every lane its
// 16-lane row sum; two row broadcasts fold the rows into lane 63.
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp<0xB1>(x);          // quad_perm [1,0,3,2]
    x += dpp<0x4E>(x);          // quad_perm [2,3,0,1]
    x += dpp<0x141>(x);         // row_half_mirror
    x += dpp<0x140>(x);         // row_mirror
    x += dpp<0x142, 0xA>(x);    // row_bcast:15 into rows 1 and 3
    x += dpp<0x143, 0xC>(x);    // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(256) void k_render_bwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                    const pg_splat* __restrict__ splats,
                                                    const int32_t* __restrict__ values,
                                                    const int2* __restrict__ ranges, float bg0, float bg1,
                                                    float bg2, const float* __restrict__ final_T,
                                                    const int32_t* __restrict__ n_contrib,
                                                    const float* __restrict__ dL_dimage, int64_t n_gv,
                                                    float* __restrict__ grad2d) {
    __shared__ float4 s_geo[BATCH];
    __shared__ float4 s_col[BATCH];
    __shared__ float s_blu[BATCH];
    __shared__ int32_t s_gv[BATCH];
    __shared__ float s_acc[9][BATCH];
    __shared__ int32_t s_maxn;
    const TileCtx c = tile_ctx<TW, TH>(views, nv, n_tiles);
    const int2 rg = ranges[c.tile];
    const float fx = (float)(c.px - (int32_t)c.ox) + 0.5f, fy = (float)(c.py - (int32_t)c.oy) + 0.5f;
    float T = 1.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
    int32_t n = 0;
    if (c.inside) {
        const int64_t HW = (int64_t)c.W * c.H;
        const int64_t vb = c.pix - ((int64_t)c.py * c.W + c.px);
        const float* gi = dL_dimage + 3 * vb + (int64_t)c.py * c.W + c.px;
        G0 = gi[0];
        G1 = gi[HW];
        G2 = gi[2 * HW];
        T = final_T[c.pix];
        n = n_contrib[c.pix];
    }
    if (threadIdx.x == 0) s_maxn = 0;
    __syncthreads();
    if (n > 0) atomicMax(&s_maxn, n);
    __syncthreads();
    const int32_t len = s_maxn;
    float B0 = bg0, B1 = bg1, B2 = bg2;
    const int lane = threadIdx.x & 63;
    for (int32_t bend = len; bend > 0; bend -= BATCH) {
        const int32_t bstart = max(0, bend - BATCH);
        const int32_t cnt = bend - bstart;
        __syncthreads();
        if ((int32_t)threadIdx.x < cnt) {
            const int32_t gv = values[rg.x + bstart + threadIdx.x];
            s_gv[threadIdx.x] = gv;
            stage(splats, gv, c.ox, c.oy, s_geo, s_col, s_blu, threadIdx.x);
        }
        for (int32_t idx = threadIdx.x; idx < 9 * BATCH; idx += 256) (&s_acc[0][0])[idx] = 0.0f;
        __syncthreads();
        for (int32_t k = cnt - 1; k >= 0; k--) {
            const float4 g = s_geo[k];
            const float dx = fx - g.x, dy = fy - g.y;
            const float4 cc = s_col[k];
            const float q = quad(dx, dy, g.z, g.w, cc.x);
            bool in = (bstart + k < n) && q <= kQMax;
            if (!__any(in)) continue;                 // wave-uniform skip
            const Eval ev = evaluate(q, cc.y);
            in = in && ev.alpha >= kAlphaMin;
            if (!__any(in)) continue;
            const float al = ev.alpha;
            const float Tk = T * __builtin_amdgcn_rcpf(1.0f - al);   // transmittance in front of k
            T = in ? Tk : T;
            const float cb = s_blu[k];
            const float w = in ? Tk * al : 0.0f;
            float v[9];
            v[6] = w * G0;
            v[7] = w * G1;
            v[8] = w * G2;
            const float dal = in ? Tk * ((G0 * (cc.z - B0) + G1 * (cc.w - B1)) + G2 * (cb - B2)) : 0.0f;
            B0 = in ? al * cc.z + (1.0f - al) * B0 : B0;
            B1 = in ? al * cc.w + (1.0f - al) * B1 : B1;
            B2 = in ? al * cb + (1.0f - al) * B2 : B2;
            const float dau = ev.raw < kAlphaMax ? dal : 0.0f;     // alpha clamped: no opacity / shape terms
            v[5] = dau * ev.e;
            const float dq = -0.5f * al * dau;
            const float bb = 0.5f * g.w;
            v[2] = dq * dx * dx;
            v[3] = dq * 2.0f * dx * dy;
            v[4] = dq * dy * dy;
            v[0] = -2.0f * dq * (g.z * dx + bb * dy);
            v[1] = -2.0f * dq * (bb * dx + cc.x * dy);
#pragma unroll
            for (int i = 0; i < 9; i++) v[i] = wave_sum(v[i]);
            if (lane == 63) {
#pragma unroll
                for (int i = 0; i < 9; i++) atomicAdd(&s_acc[i][k], v[i]);
            }
        }
        __syncthreads();
        for (int32_t idx = threadIdx.x; idx < 9 * cnt; idx += 256) {
            const int32_t i = idx / cnt, k = idx - i * cnt;
            const float val = s_acc[i][k];
            if (val != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)i * n_gv + s_gv[k]], val);
        }
    }
}

template <int TW, int TH, int BATCH>
void fwd_launch(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* ranges,
                const float bg[3], float* image, float* final_T, int32_t* n_contrib, uint64_t* counters,
                hipStream_t s) {
    const unsigned grid = (unsigned)v->n_tiles;
    if (counters)
        k_render_fwd<TW, TH, BATCH, true><<<grid, 256, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), bg[0], bg[1],
            bg[2], image, final_T, n_contrib, reinterpret_cast<unsigned long long*>(counters));
    else
        k_render_fwd<TW, TH, BATCH, false><<<grid, 256, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), bg[0], bg[1],
            bg[2], image, final_T, n_contrib, nullptr);
}

template <int TW, int TH, int BATCH>
void bwd_launch(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* ranges,
                const float bg[3], const float* final_T, const int32_t* n_contrib, const float* dL_dimage,
                float* grad2d, hipStream_t s) {
    k_render_bwd<TW, TH, BATCH><<<(unsigned)v->n_tiles, 256, 0, s>>>(
        v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), bg[0], bg[1],
        bg[2], final_T, n_contrib, dL_dimage, v->n_gv, grad2d);
}

template <template <int, int, int> class F, typename... A>
void dispatch(const pg_tiling& t, A... a) {
    const int b = t.lds_batch;
    if (t.tile_w == 16) {
        if (b == 64) F<16, 16, 64>::run(a...); else if (b == 128) F<16, 16, 128>::run(a...); else F<16, 16, 256>::run(a...);
    } else if (t.tile_w == 8) {
        if (b == 64) F<8, 32, 64>::run(a...); else if (b == 128) F<8, 32, 128>::run(a...); else F<8, 32, 256>::run(a...);
    } else {
        if (b == 64) F<32, 8, 64>::run(a...); else if (b == 128) F<32, 8, 128>::run(a...); else F<32, 8, 256>::run(a...);
    }
}

template <int TW, int TH, int B>
struct FwdRun {
    template <typename... A>
    static void run(A... a) { fwd_launch<TW, TH, B>(a...); }
};
template <int TW, int TH, int B>
struct BwdRun {
    template <typename... A>
    static void run(A... a) { bwd_launch<TW, TH, B>(a...); }
};

}  // namespace

hipError_t launch_render_fwd(const pg_views* v, const pg_splat* splats, const int32_t* values,
                             const int32_t* ranges, const float bg[3], float* image, float* final_T,
                             int32_t* n_contrib, uint64_t* counters, hipStream_t s) {
    if (v->n_tiles == 0) return hipSuccess;
    dispatch<FwdRun>(v->tiling, v, splats, values, ranges, bg, image, final_T, n_contrib, counters, s);
    return hipGetLastError();
}

hipError_t launch_render_bwd(const pg_views* v, const pg_splat* splats, const int32_t* values,
                             const int32_t* ranges, const float bg[3], const float* final_T,
                             const int32_t* n_contrib, const float* dL_dimage, float* grad2d, hipStream_t s) {
    hipError_t e = fill_u32(grad2d, 0u, 9 * v->n_gv, s);
    if (e != hipSuccess || v->n_tiles == 0) return e;
    dispatch<BwdRun>(v->tiling, v, splats, values, ranges, bg, final_T, n_contrib, dL_dimage, grad2d, s);
    return hipGetLastError();
}

}  // namespace pg
