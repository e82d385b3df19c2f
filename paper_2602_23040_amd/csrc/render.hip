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

// One wave (64 lanes) composites one tile; lane l owns the four pixels
// l, l + 64, l + 128, l + 192 of the tile in row-major order, so each group
// of 64 pixels ("slot") is a 64-lane sub-block of the tile.  Every staged
// Gaussian is read from LDS once per lane and applied to four pixels, and the
// adjoint needs one cross-lane reduction per Gaussian and tile instead of one
// per 64 pixels.  A slot whose 64 pixels all miss the ellipse is skipped with
// a wave-uniform branch.
constexpr int kLanes = 64;
constexpr int kPPT = 4;

struct TileGeo {
    int64_t tile, vbase;
    int32_t W, H;
    double ox, oy;
    int32_t px[kPPT], py[kPPT];
    float fx[kPPT], fy[kPPT];
    bool inside[kPPT];
};

template <int TW, int TH>
__device__ __forceinline__ void tile_geo(const ViewDev* views, int nv, int64_t n_tiles, TileGeo& t) {
    t.tile = xcd_remap(blockIdx.x, n_tiles);
    const int v = find_view_by_tile(views, nv, t.tile);
    const ViewDev& V = views[v];
    const int64_t lt = t.tile - V.tile_base;
    const int32_t tx = (int32_t)(lt % V.TX), ty = (int32_t)(lt / V.TX);
    t.W = V.W;
    t.H = V.H;
    t.vbase = V.pix_base;
    const int32_t ox = (tx * TW) & ~31, oy = (ty * TH) & ~31;
    t.ox = (double)ox;
    t.oy = (double)oy;
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        const int32_t lp = (int32_t)threadIdx.x + kLanes * j;
        t.px[j] = tx * TW + lp % TW;
        t.py[j] = ty * TH + lp / TW;
        t.fx[j] = (float)(t.px[j] - ox) + 0.5f;
        t.fy[j] = (float)(t.py[j] - oy) + 0.5f;
        t.inside[j] = t.px[j] < t.W && t.py[j] < t.H;
    }
}

// Stage Gaussian `gv` into LDS slot `k` in coordinates local to (ox, oy).
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
__global__ __launch_bounds__(kLanes) void k_render_fwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                       const pg_splat* __restrict__ splats,
                                                       const int32_t* __restrict__ values,
                                                       const int2* __restrict__ ranges, float bg0, float bg1,
                                                       float bg2, float* __restrict__ image,
                                                       float* __restrict__ final_T, int32_t* __restrict__ n_contrib,
                                                       unsigned long long* __restrict__ counters) {
    __shared__ float4 s_geo[BATCH];
    __shared__ float4 s_col[BATCH];
    __shared__ float s_blu[BATCH];
    TileGeo t;
    tile_geo<TW, TH>(views, nv, n_tiles, t);
    const int2 rg = ranges[t.tile];
    float T[kPPT], C0[kPPT], C1[kPPT], C2[kPPT];
    int32_t n[kPPT];
    bool done[kPPT];
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        T[j] = 1.0f;
        C0[j] = C1[j] = C2[j] = 0.0f;
        n[j] = 0;
        done[j] = !t.inside[j];
    }
    uint32_t n_eval = 0, n_comp = 0;
    for (int32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
        bool alive = false;
#pragma unroll
        for (int j = 0; j < kPPT; j++) alive = alive || !done[j];
        if (!__any(alive)) break;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < BATCH && b0 + i < rg.y; i += kLanes)
            stage(splats, values[b0 + i], t.ox, t.oy, s_geo, s_col, s_blu, i);
        __syncthreads();
        const int32_t cnt = min(BATCH, rg.y - b0);
        for (int32_t k = 0; k < cnt; k++) {
            const float4 g = s_geo[k];
            const float4 cc = s_col[k];
            const float cb = s_blu[k];
            const int32_t pos1 = b0 - rg.x + k + 1;
#pragma unroll
            for (int j = 0; j < kPPT; j++) {
                const float dx = t.fx[j] - g.x, dy = t.fy[j] - g.y;
                const float q = quad(dx, dy, g.z, g.w, cc.x);
                if (STATS) n_eval += done[j] ? 0u : 1u;
                bool in = !done[j] && q <= kQMax;
                if (!__any(in)) continue;             // wave-uniform: no pixel of this slot inside
                const Eval ev = evaluate(q, cc.y);
                in = in && ev.alpha >= kAlphaMin;
                const float Tn = T[j] * (1.0f - ev.alpha);
                const bool stop = in && Tn < kTMin;
                const bool take = in && !stop;
                done[j] = done[j] || stop;
                const float w = take ? T[j] * ev.alpha : 0.0f;
                C0[j] = fmaf(w, cc.z, C0[j]);
                C1[j] = fmaf(w, cc.w, C1[j]);
                C2[j] = fmaf(w, cb, C2[j]);
                T[j] = take ? Tn : T[j];
                n[j] = take ? pos1 : n[j];
                if (STATS) n_comp += take ? 1u : 0u;
            }
            bool alive2 = false;
#pragma unroll
            for (int j = 0; j < kPPT; j++) alive2 = alive2 || !done[j];
            if (!__any(alive2)) break;                // every pixel of the tile has terminated
        }
    }
    const int64_t HW = (int64_t)t.W * t.H;
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        if (!t.inside[j]) continue;
        const int64_t p = (int64_t)t.py[j] * t.W + t.px[j];
        float* img = image + 3 * t.vbase + p;
        img[0] = fmaf(T[j], bg0, C0[j]);
        img[HW] = fmaf(T[j], bg1, C1[j]);
        img[2 * HW] = fmaf(T[j], bg2, C2[j]);
        final_T[t.vbase + p] = T[j];
        n_contrib[t.vbase + p] = n[j];
    }
    if (STATS) {
        unsigned long long e = n_eval, c = n_comp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if (threadIdx.x == 0) {
            atomicAdd(&counters[0], e);
            atomicAdd(&counters[1], c);
        }
    }
}

// Cross-lane data-parallel-primitive move: lanes of disabled rows read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Sums of N values over the 64 lanes of the wave with DPP moves only (no LDS
// traffic), the N reductions interleaved step by step: butterflies inside
// quads, half-row and row mirrors give every lane its 16-lane row sum, two row
// broadcasts fold the rows into lane 63, which is read into a scalar.
template <int N>
__device__ __forceinline__ void wave_sums(float* x) {
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0xB1>(x[i]);          // quad_perm [1,0,3,2]
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0x4E>(x[i]);          // quad_perm [2,3,0,1]
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0x141>(x[i]);         // row_half_mirror
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0x140>(x[i]);         // row_mirror
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0x142, 0xA>(x[i]);    // row_bcast:15 into rows 1, 3
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp<0x143, 0xC>(x[i]);    // row_bcast:31 into rows 2, 3
#pragma unroll
    for (int i = 0; i < N; i++) x[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[i]), 63));
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(kLanes) void k_render_bwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
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
    TileGeo t;
    tile_geo<TW, TH>(views, nv, n_tiles, t);
    const int2 rg = ranges[t.tile];
    const int64_t HW = (int64_t)t.W * t.H;
    float T[kPPT], G0[kPPT], G1[kPPT], G2[kPPT], B0[kPPT], B1[kPPT], B2[kPPT];
    int32_t n[kPPT];
    int32_t maxn = 0;
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        T[j] = 1.0f;
        G0[j] = G1[j] = G2[j] = 0.0f;
        B0[j] = bg0;
        B1[j] = bg1;
        B2[j] = bg2;
        n[j] = 0;
        if (t.inside[j]) {
            const int64_t p = (int64_t)t.py[j] * t.W + t.px[j];
            const float* gi = dL_dimage + 3 * t.vbase + p;
            G0[j] = gi[0];
            G1[j] = gi[HW];
            G2[j] = gi[2 * HW];
            T[j] = final_T[t.vbase + p];
            n[j] = n_contrib[t.vbase + p];
        }
        maxn = max(maxn, n[j]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, __shfl_xor(maxn, o, 64));
    const int lane = threadIdx.x;
    for (int32_t bend = maxn; bend > 0; bend -= BATCH) {
        const int32_t bstart = max(0, bend - BATCH);
        const int32_t cnt = bend - bstart;
        __syncthreads();
        for (int32_t i = lane; i < cnt; i += kLanes) {
            const int32_t gv = values[rg.x + bstart + i];
            s_gv[i] = gv;
            stage(splats, gv, t.ox, t.oy, s_geo, s_col, s_blu, i);
        }
        __syncthreads();
        for (int32_t k = cnt - 1; k >= 0; k--) {
            const float4 g = s_geo[k];
            const float4 cc = s_col[k];
            const float cb = s_blu[k];
            const float bb = 0.5f * g.w;
            const int32_t pos = bstart + k;
            float acc[9];
#pragma unroll
            for (int i = 0; i < 9; i++) acc[i] = 0.0f;
            bool any_c = false;
#pragma unroll
            for (int j = 0; j < kPPT; j++) {
                const float dx = t.fx[j] - g.x, dy = t.fy[j] - g.y;
                const float q = quad(dx, dy, g.z, g.w, cc.x);
                bool in = pos < n[j] && q <= kQMax;
                if (!__any(in)) continue;             // wave-uniform skip
                const Eval ev = evaluate(q, cc.y);
                in = in && ev.alpha >= kAlphaMin;
                if (!__any(in)) continue;
                any_c = true;
                const float al = ev.alpha;
                const float Tk = T[j] * __builtin_amdgcn_rcpf(1.0f - al);   // transmittance in front of k
                T[j] = in ? Tk : T[j];
                const float w = in ? Tk * al : 0.0f;
                acc[6] += w * G0[j];
                acc[7] += w * G1[j];
                acc[8] += w * G2[j];
                const float dal =
                    in ? Tk * ((G0[j] * (cc.z - B0[j]) + G1[j] * (cc.w - B1[j])) + G2[j] * (cb - B2[j])) : 0.0f;
                B0[j] = in ? al * cc.z + (1.0f - al) * B0[j] : B0[j];
                B1[j] = in ? al * cc.w + (1.0f - al) * B1[j] : B1[j];
                B2[j] = in ? al * cb + (1.0f - al) * B2[j] : B2[j];
                const float dau = ev.raw < kAlphaMax ? dal : 0.0f;   // clamped alpha: no opacity / shape terms
                acc[5] += dau * ev.e;
                const float dq = -0.5f * al * dau;
                acc[2] += dq * dx * dx;
                acc[3] += dq * 2.0f * dx * dy;
                acc[4] += dq * dy * dy;
                acc[0] += -2.0f * dq * (g.z * dx + bb * dy);
                acc[1] += -2.0f * dq * (bb * dx + cc.x * dy);
            }
            if (!any_c) continue;
            wave_sums<9>(acc);
            float mine = 0.0f;
#pragma unroll
            for (int i = 0; i < 9; i++) mine = (lane == i) ? acc[i] : mine;
            if (lane < 9) unsafeAtomicAdd(&grad2d[(int64_t)lane * n_gv + s_gv[k]], mine);
        }
    }
}

template <int TW, int TH, int BATCH>
void fwd_launch(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* ranges,
                const float bg[3], float* image, float* final_T, int32_t* n_contrib, uint64_t* counters,
                hipStream_t s) {
    const unsigned grid = (unsigned)v->n_tiles;
    if (counters)
        k_render_fwd<TW, TH, BATCH, true><<<grid, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), bg[0], bg[1],
            bg[2], image, final_T, n_contrib, reinterpret_cast<unsigned long long*>(counters));
    else
        k_render_fwd<TW, TH, BATCH, false><<<grid, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), bg[0], bg[1],
            bg[2], image, final_T, n_contrib, nullptr);
}

template <int TW, int TH, int BATCH>
void bwd_launch(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* ranges,
                const float bg[3], const float* final_T, const int32_t* n_contrib, const float* dL_dimage,
                float* grad2d, hipStream_t s) {
    k_render_bwd<TW, TH, BATCH><<<(unsigned)v->n_tiles, kLanes, 0, s>>>(
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
