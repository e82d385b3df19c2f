// a4 -- front-to-back compositing per screen tile, and (a5, first half) its
// adjoint per pixel; the adjoint takes the image cotangent as given, or forms
// the L1 term's (Sec. 4.2 "Objective") from image and target itself.
//
// Compositing follows C = sum_i T_i alpha_i c_i with T_i = prod_{j<i}
// (1 - alpha_j) (supplementary, viewer section), restricted to the 3-sigma
// ellipse q = d^2 <= 9 of Sec. 4.2; alpha = min(0.99, o e^{-q/2}), Gaussians
// with alpha < 1/255 are skipped, and a pixel stops before the Gaussian that
// would bring T below 1e-4.
//
// Launch shape: one wave64 work-group per (view, tile) of 256 pixels, four
// pixels per lane.  The tile is four 8x8 blocks (2x2 for 16x16 tiles, 1x4 for
// 8x32, 4x1 for 32x8); lane l holds pixel (l % 8, l / 8) of every block.  The
// tile's list is staged through LDS in batches of BATCH Gaussians (one
// gathered 48-byte record each) and every lane reads each staged Gaussian as
// an LDS broadcast, so the loop is bound by FP32 VALU work, not HBM.  Blocks
// that a Gaussian's conservative x/y extent misses, or whose pixels have all
// terminated, are skipped wave-uniformly (ballots), and the tile stops once
// every pixel has terminated.  Work-groups are assigned so that consecutive
// tiles run on the same XCD (the dispatcher deals groups round-robin over the
// 8 XCDs), which keeps the records neighbouring tiles share in one L2.
// When the sort's tile dispatch order is given, work-group b takes the b-th
// tile of that order instead (longest lists first, which shortens the tail
// of the launch more than the shared L2 saves).
//
// Pixel offsets are formed in FP32 coordinates local to the 32x32 pixel block
// holding the tile (every supported tile shape nests in such a block), from
// the FP64 pixel-space mean: q keeps full FP32 precision at 1080p, and a
// pixel sees bit-identical inputs whatever the tile shape.
//
// The forward records, per tile, one 32-bit word per Gaussian that composited
// at least one pixel: its list position and the blocks where it did.  While
// 64 Gaussians are composited, one scalar bit mask per block collects which
// of them were taken; lane i then forms the word of Gaussian i and the words
// are stored compacted and coalesced.  The adjoint walks only those entries,
// back to front.  n_contrib is the list position at which the pixel stopped
// (the Gaussian that would have brought T below 1e-4), or the list length if
// it never did; until then a pixel takes every Gaussian with q <= 9 and
// alpha >= 1/255.  So a pixel took entry k exactly when k is below its
// n_contrib and both tests pass, and q and alpha are recomputed by the same
// code as the forward, so the
// adjoint's decisions are the forward's.  The transmittance in front of
// Gaussian k is recovered as T_k = T_{k+1} / (1 - alpha_k) from the stored
// final T (no per-step storage).  Per-Gaussian sums over the tile's pixels
// are reduced across the wave with DPP / permlane moves, two consecutive
// entries at a time (they share the exchange steps), and written, without
// atomics, to the (Gaussian, tile) instance's own slot, tagged with the
// sort's generation; the projection adjoint then adds the slots of each
// (view, Gaussian) in a fixed order, counting only slots of the current
// generation (instances that composited nothing keep an older tag and read as
// zero, so the slots are never cleared), and gradients are bitwise
// deterministic.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr float kQMax = 9.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
// The staged conic is scaled by -log2(e) / 2, so the quadratic form gives
// s = -q log2(e) / 2 directly: e^{-q/2} = 2^s, and q <= 9 reads s >= 9 (-log2(e) / 2).
// The opacity is staged as lo = log2 o and added in the quadratic's last
// fused multiply-add: s' = s + lo, and o e^{-q/2} = 2^{s'} without a multiply.
constexpr float kQScale = -0.72134752044448170f;
constexpr float kSMin = kQMax * kQScale;
constexpr float kLog2AlphaMin = -7.99435343685885793f;     // log2(1 / 255)
constexpr float kLog2AlphaMax = -0.01449956969511509f;     // log2(0.99)

// The one definition of s', alpha and the take decision used by both the
// forward and the adjoint, with explicit fused multiply-adds so both kernels
// take bit-identical decisions (the library is compiled with -ffp-contract=off).
__device__ __forceinline__ float quad(float dx, float dy, float a, float b2, float c, float lo) {
    const float u = fmaf(b2, dy, a * dx);      // a dx + 2 b dy
    return fmaf(u, dx, fmaf(c, dy * dy, lo));  // dx (a dx + 2 b dy) + c dy^2 + lo
}

// Smallest s' a pixel needs: q <= 9 (s' >= kSMin + lo) and alpha >= 1/255
// (s' >= log2(1/255)); one compare per pixel.  log2 o = -inf (o = 0) or NaN
// (o < 0) makes s' -inf or NaN, which no pixel passes.
__device__ __forceinline__ float take_threshold(float lo) {
    return fmaxf(kSMin + lo, kLog2AlphaMin);
}

// The 0.99 clamp can only bind when lo >= log2(0.99), since 2^{s'} <= 2^{lo}
// for q >= 0: the flag is decided per Gaussian (as integer bits, the same in
// both kernels; lo <= 0, and lo = 0 for o = 1).  The forward clamps at a cap
// (0.99, or +inf when the flag is clear: one median either way); the adjoint
// has a copy of its loop without the clamp for the Gaussians that cannot
// reach it, and takes alpha = 2^{s'} there, the forward's value for every
// non-NaN s'.
__device__ __forceinline__ bool may_clamp(float lo) {
    const int b = __float_as_int(lo);
    return b >= 0 || b <= __float_as_int(kLog2AlphaMax);
}

__device__ __forceinline__ float raw_alpha(float s1) {
    return __builtin_amdgcn_exp2f(s1);                    // o e^{-q/2}
}

// min(raw, cap) for the raw >= 0 of every pixel that can take the Gaussian
// (its opacity is positive): one median, with no NaN canonicalisation of cap
__device__ __forceinline__ float clamp_alpha(float raw, float cap) {
    return __builtin_amdgcn_fmed3f(raw, 0.0f, cap);
}

__device__ __forceinline__ int64_t xcd_remap(int64_t i, int64_t n) {
    const int64_t per = n >> 3, rem = n & 7;
    const int64_t x = i & 7, j = i >> 3;
    return x * per + imin(x, rem) + j;
}

// One wave (64 lanes) composites one tile of 256 pixels, seen as four 8x8
// pixel blocks ("slots": 2x2 blocks for 16x16 tiles, 1x4 for 8x32, 4x1 for
// 32x8).  Lane l owns pixel (l % 8, l / 8) of every block.  Every staged
// Gaussian is read from LDS once per lane and applied to four pixels; the
// adjoint needs one cross-lane reduction per Gaussian and tile; a block the
// ellipse cannot reach is skipped with a scalar branch.
constexpr int kLanes = 64;
constexpr int kPPT = 4;

struct TileGeo {
    int64_t tile, vbase;
    int32_t tx, ty;
    int32_t W, H;
    double ox, oy;
    float col0, row0;            // local x, y of the tile's first pixel
    int32_t px[kPPT], py[kPPT];
    float fx[kPPT], fy[kPPT];
    bool inside[kPPT];
};

// False when the dispatch order names no valid tile (the work-group then exits).
template <int TW, int TH>
__device__ __forceinline__ bool tile_geo(const ViewDev* views, int nv, int64_t n_tiles, const int32_t* order,
                                         TileGeo& t) {
    t.tile = order ? (int64_t)__builtin_amdgcn_readfirstlane(order[blockIdx.x]) : xcd_remap(blockIdx.x, n_tiles);
    if (t.tile < 0 || t.tile >= n_tiles) return false;
    const int v = find_view_by_tile(views, nv, t.tile);
    const ViewDev& V = views[v];
    const int64_t lt = t.tile - V.tile_base;
    const int32_t tx = (int32_t)(lt % V.TX), ty = (int32_t)(lt / V.TX);
    t.tx = tx;
    t.ty = ty;
    t.W = V.W;
    t.H = V.H;
    t.vbase = V.pix_base;
    const int32_t ox = (tx * TW) & ~31, oy = (ty * TH) & ~31;
    t.ox = (double)ox;
    t.oy = (double)oy;
    t.col0 = (float)(tx * TW - ox);
    t.row0 = (float)(ty * TH - oy);
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        constexpr int BPR = TW / 8;              // 8x8 blocks per tile row
        t.px[j] = tx * TW + (j % BPR) * 8 + (int32_t)threadIdx.x % 8;
        t.py[j] = ty * TH + (j / BPR) * 8 + (int32_t)threadIdx.x / 8;
        t.fx[j] = (float)(t.px[j] - ox) + 0.5f;
        t.fy[j] = (float)(t.py[j] - oy) + 0.5f;
        t.inside[j] = t.px[j] < t.W && t.py[j] < t.H;
    }
    return true;
}

// Stage Gaussian `gv` into LDS slot `k` in coordinates local to (ox, oy) and,
// when MASK is set, the mask of 8x8 pixel blocks its ellipse q <= 9 can reach:
// blocks whose pixel-centre rectangle meets the ellipse's bounding box, with
// half-extents 3 sqrt(Sigma_xx) and 3 sqrt(Sigma_yy), (Sigma_xx, Sigma_yy) =
// (c, a) / (a c - b^2) from the conic.  The bounds are widened (0.1% +
// 0.01 px) to cover FP32 rounding of q and fall back to "all blocks" for
// ill-conditioned conics, so a skipped block never holds a pixel with q <= 9
// and results are unchanged.  (Testing the minimum of q over each block
// rectangle instead cost more at staging than it saved.)
// One staged Gaussian in LDS: one record per list entry, so a wave reads all
// of it from a single address register with immediate offsets.  aux holds the
// block mask (forward) or the gradient slot and the entry word (adjoint).
struct alignas(16) Staged {
    float4 geo;          // local mean x, y; conic a, 2 b (scaled by kQScale)
    float4 col;          // conic c (scaled by kQScale), log2 opacity, red, green
    float blu;           // blue
    float thr;           // take_threshold(log2 opacity)
    uint32_t aux[2];
};

constexpr uint32_t kClampBit = 1u << kPPT;   // forward's aux[0]: may_clamp(log2 opacity)
// adjoint's aux[0]: the gradient slot (kNoSlot: none) and, in bit 31, may_clamp(log2 opacity)
constexpr uint32_t kNoSlot = 0x7fffffffu;
constexpr uint32_t kSlotClamp = 0x80000000u;

template <int TW, int TH, bool MASK>
__device__ __forceinline__ float stage(const pg_splat* __restrict__ splats, int32_t gv, double ox, double oy,
                                      float col0, float row0, Staged* s_st, int k) {
    const float4* sp = reinterpret_cast<const float4*>(splats + gv);
    const float4 a = sp[0], b = sp[1], c = sp[2];
    double2 m;
    *reinterpret_cast<float4*>(&m) = a;
    const float mx = (float)(m.x - ox), my = (float)(m.y - oy);
    s_st[k].geo = make_float4(mx, my, b.x * kQScale, 2.0f * b.y * kQScale);
    const float lo = __builtin_amdgcn_logf(b.w);                // log2 opacity
    s_st[k].col = make_float4(b.z * kQScale, lo, c.x, c.y);     // scaled conic c, log2 opacity, red, green
    s_st[k].blu = c.z;
    s_st[k].thr = take_threshold(lo);
    if (!MASK) return lo;
    constexpr int BPR = TW / 8;
    const float ac = b.x * b.z;
    const float det = ac - b.y * b.y;
    uint32_t mask = (1u << kPPT) - 1u;
    if (det > 1e-2f * ac && b.x > 0.0f && b.z > 0.0f) {
        const float ex = 3.0f * sqrtf(b.z / det) * 1.001f + 0.01f;
        const float ey = 3.0f * sqrtf(b.x / det) * 1.001f + 0.01f;
        mask = 0u;
#pragma unroll
        for (int j = 0; j < kPPT; j++) {
            const float x0 = col0 + (float)((j % BPR) * 8) + 0.5f, y0 = row0 + (float)((j / BPR) * 8) + 0.5f;
            if (mx + ex >= x0 && mx - ex <= x0 + 7.0f && my + ey >= y0 && my - ey <= y0 + 7.0f) mask |= 1u << j;
        }
    }
    s_st[k].aux[0] = mask | (may_clamp(lo) ? kClampBit : 0u);
    return lo;
}

// Eight waves per SIMD (64 registers): the forward waits on its per-Gaussian
// LDS reads between short VALU runs, and the eighth wave hides more of that
// (2.13 -> 2.08 ms on 50 views); the adjoint stays at seven, where eight would spill.
template <int TW, int TH, int BATCH, bool STATS>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_render_fwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                       const pg_splat* __restrict__ splats,
                                                       const int32_t* __restrict__ values,
                                                       const int2* __restrict__ ranges,
                                                       const int32_t* __restrict__ order, float bg0, float bg1,
                                                       float bg2, float* __restrict__ image,
                                                       float* __restrict__ final_T, int32_t* __restrict__ n_contrib,
                                                       int32_t* __restrict__ tile_entries,
                                                       uint32_t* __restrict__ entries,
                                                       unsigned long long* __restrict__ counters) {
    __shared__ Staged s_st[BATCH];     // aux[0]: the mask of 8x8 blocks the ellipse can reach, kClampBit
    TileGeo t;
    if (!tile_geo<TW, TH>(views, nv, n_tiles, order, t)) return;
    const int2 rg = ranges[t.tile];
    float T[kPPT], C0[kPPT], C1[kPPT], C2[kPPT];
    int32_t n[kPPT];         // list positions the pixel reached: where it stopped, else the list length
    uint64_t live[kPPT];     // lanes of slot j still compositing (wave-uniform lane mask)
    uint32_t alive = 0;      // bit j: live[j] != 0 (one scalar test per block instead of a 64-bit one)
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        T[j] = 1.0f;
        C0[j] = C1[j] = C2[j] = 0.0f;
        n[j] = rg.y - rg.x;
        live[j] = __ballot(t.inside[j]);
        alive |= live[j] != 0 ? 1u << j : 0u;
    }
    uint64_t n_eval = 0, n_comp = 0;        // wave totals (STATS only)
    int32_t n_entries = 0;                  // Gaussians of the tile list that composited somewhere
    const int lane = threadIdx.x;
    for (int32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
        if (alive == 0) break;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < BATCH && b0 + i < rg.y; i += kLanes)
            stage<TW, TH, true>(splats, values[b0 + i], t.ox, t.oy, t.col0, t.row0, s_st, i);
        __syncthreads();
        const int32_t cnt = min(BATCH, rg.y - b0);
        // sub-batches of 64 Gaussians: bit (k - k0) of took[j] records that a pixel of block j took Gaussian k
        for (int32_t k0 = 0; k0 < cnt && alive != 0; k0 += kLanes) {
            const int32_t k1 = min(cnt, k0 + kLanes);
            uint64_t took[kPPT] = {0, 0, 0, 0};
            // one Gaussian of the sub-batch (two per loop iteration: the loop and
            // liveness bookkeeping is shared)
            auto gauss = [&](const int32_t k) __attribute__((always_inline)) {
                const float4 g = s_st[k].geo;
                const float4 cc = s_st[k].col;
                const float cb = s_st[k].blu;
                const float thr = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_st[k].thr)));
                // wave-uniform: block bits and the clamp flag, tested on the scalar unit
                const uint32_t mask = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_st[k].aux[0]);
                const int32_t pos = b0 - rg.x + k;
                const uint64_t kbit = 1ull << (k - k0);
                // selected as integer bits, so the select stays on the scalar unit
                const float cap = __int_as_float((mask & kClampBit) ? __float_as_int(kAlphaMax) : 0x7f800000);
                const uint32_t act = mask & alive;    // blocks the ellipse can reach that still composite
#pragma unroll
                for (int j = 0; j < kPPT; j++) {
                    if (STATS) n_eval += __popcll(live[j]);
                    if (!((act >> j) & 1u)) continue;   // ellipse misses the block / block done
                    const float dx = t.fx[j] - g.x, dy = t.fy[j] - g.y;
                    const float qs = quad(dx, dy, g.z, g.w, cc.x, cc.y);   // -q log2(e) / 2 + log2 o
                    const uint64_t inm = __ballot(qs >= thr) & live[j];   // q <= 9 and alpha >= 1/255
                    if (inm == 0) continue;
                    const float alpha = clamp_alpha(raw_alpha(qs), cap);
                    const float wa = T[j] * alpha;
                    const float Tn = T[j] - wa;          // T (1 - alpha)
                    const uint64_t stopm = __ballot(Tn < kTMin) & inm;
                    const uint64_t takem = inm & ~stopm;
                    if (stopm) {     // once per pixel
                        live[j] &= ~stopm;
                        n[j] = __builtin_amdgcn_inverse_ballot_w64(stopm) ? pos : n[j];
                        if (live[j] == 0) alive &= ~(1u << j);
                    }
                    took[j] |= takem ? kbit : 0ull;
                    if (STATS) n_comp += __popcll(takem);
                    const bool take = __builtin_amdgcn_inverse_ballot_w64(takem);
                    const float w = take ? wa : 0.0f;
                    C0[j] = fmaf(w, cc.z, C0[j]);
                    C1[j] = fmaf(w, cc.w, C1[j]);
                    C2[j] = fmaf(w, cb, C2[j]);
                    T[j] = take ? Tn : T[j];
                }
            };
            for (int32_t k = k0; k < k1; k += 2) {
                gauss(k);
                if (alive == 0) break;   // every pixel has terminated
                if (k + 1 < k1) {
                    gauss(k + 1);
                    if (alive == 0) break;
                }
            }
            // entries of the sub-batch for the adjoint (lane i: Gaussian k0 + i), stored in list order
            uint32_t bits = 0;
#pragma unroll
            for (int j = 0; j < kPPT; j++) bits |= (uint32_t)((took[j] >> lane) & 1ull) << j;
            const uint64_t em = __ballot(bits != 0);
            const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(em >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)em, 0u));
            if (bits != 0) entries[rg.x + n_entries + (int32_t)before] = ((uint32_t)(b0 - rg.x + k0 + lane) << 4) | bits;
            n_entries += __popcll(em);
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
    if (lane == 0) tile_entries[t.tile] = n_entries;
    if (STATS && threadIdx.x == 0) {
        atomicAdd(&counters[0], (unsigned long long)n_eval);
        atomicAdd(&counters[1], (unsigned long long)n_comp);
    }
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return dpp_f32<CTRL, ROW_MASK>(v);
}

// Cross-wave totals of the nine per-lane sums of two consecutive entries
// (A, B), with the gfx950 register swaps and DPP moves; no LDS traffic.
//  1. Row swaps: a row swap of two registers a, b followed by an add leaves
//     rows (a0+a1, b0+b1, a2+a3, b2+b3), and a half-wave swap of two such
//     registers then leaves one register whose row r holds value r summed over
//     the four rows.  Each entry's first eight sums become two such registers
//     (values 0-3 and 4-7, one per row) as soon as the entry is done; the two
//     ninth sums share one register (rows 0 and 1).
//  2. Inside the rows, four exchange steps (lane xor 1, xor 2, rotate by 4 and
//     by 8) finish the sums.  At the first three, two registers are merged:
//     each lane keeps one operand and adds the partner lane's other operand,
//     so a register's values occupy half as many lanes after each step and
//     the five registers end as one.
// Result: lane 16 r + 0 / + 1 hold A's totals r / 4 + r, lanes 16 r + 2 / + 3
// B's, lane 4 A's ninth and lane 20 B's ninth (see pair_offsets).
__device__ __forceinline__ float swap16_sum(float a, float b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap32_sum(float a, float b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// lane keeps p where sel is false and q where it is true, summed with the partner lane's copy
template <int CTRL>
__device__ __forceinline__ float merge(float p, float q, bool sel) {
    return (sel ? q : p) + dpp<CTRL>(sel ? p : q);
}

struct RowSums {
    float lo, hi;        // values 0-3 and 4-7 of one entry, one per row
};
__device__ __forceinline__ RowSums row_sums(const float* v) {
    return {swap32_sum(swap16_sum(v[0], v[1]), swap16_sum(v[2], v[3])),
            swap32_sum(swap16_sum(v[4], v[5]), swap16_sum(v[6], v[7]))};
}

__device__ __forceinline__ float pair_totals(RowSums a, float a8, RowSums b, float b8, int lane) {
    const float n = swap32_sum(swap16_sum(a8, b8), 0.0f);          // rows: A's ninth, B's ninth, 0, 0
    const float ma = merge<0xB1>(a.lo, a.hi, lane & 1);             // quad_perm [1,0,3,2]
    const float mb = merge<0xB1>(b.lo, b.hi, lane & 1);
    const float n1 = n + dpp<0xB1>(n);
    const float m = merge<0x4E>(ma, mb, lane & 2);                  // quad_perm [2,3,0,1]
    const float n2 = n1 + dpp<0x4E>(n1);
    const float t = merge<0x124>(m, n2, lane & 4);                  // row_ror:4
    // row_ror:8 (every lane has a source, so bound_ctrl changes nothing; it lets
    // the move fold into the add)
    return t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x128, 0xf, 0xf, true));
}

// Byte offsets, in A's and B's 40-byte slots, of the word this lane stores
// after pair_totals: a total, the generation tag (lanes 8 and 24 hold no total
// of their entry), or 40 (outside the slot: nothing is stored).
__device__ __forceinline__ void pair_offsets(int lane, int& offA, int& offB) {
    const int p = lane & 15, r = lane >> 4;
    const int tag = 4 * (kSlotWords - 1), none = 4 * kSlotWords;
    offA = p == 0 ? 4 * r : (p == 1 ? 4 * (4 + r) : (lane == 4 ? 32 : (lane == 8 ? tag : none)));
    offB = p == 2 ? 4 * r : (p == 3 ? 4 * (4 + r) : (lane == 20 ? 32 : (lane == 24 ? tag : none)));
}

// L1: the cotangent is the L1 term's, sign(image - target) / n per channel
// (the expression of the L1 loss kernel, so bitwise its values), formed from
// image and target as the tile starts; the tile's sum of |image - target|
// (FP32 inside each row of 16 lanes, the four rows in FP64; a fixed order)
// goes to tile_loss[tile] for the loss value.
// Seven waves per SIMD: the hint holds the register allocation at 72.
template <int TW, int TH, int BATCH, bool L1>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(7))) void k_render_bwd(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                       const pg_splat* __restrict__ splats,
                                                       const pg_tile_set* __restrict__ tiles,
                                                       const int32_t* __restrict__ values,
                                                       const int2* __restrict__ ranges,
                                                       const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ inst_first,
                                                       const int32_t* __restrict__ tile_entries,
                                                       const uint32_t* __restrict__ entries,
                                                       const int32_t* __restrict__ n_contrib, float bg0,
                                                       float bg1, float bg2, const float* __restrict__ final_T,
                                                       const float* __restrict__ dL_dimage,
                                                       const int64_t* __restrict__ n_inst_dev, int64_t cap,
                                                       float* __restrict__ inst_grad, const float* __restrict__ image,
                                                       const float* __restrict__ target, float inv_n,
                                                       double* __restrict__ tile_loss) {
    // aux[0]: gradient slot of the (Gaussian, this tile) instance (kNoSlot: none) | kSlotClamp;
    // aux[1]: entry word, list position << 4 | blocks that composited it
    __shared__ Staged s_st[BATCH];
    TileGeo t;
    if (!tile_geo<TW, TH>(views, nv, n_tiles, order, t)) return;
    const int64_t HW = (int64_t)t.W * t.H;
    // Per pixel: T, the colour cotangent G, and S = G . B, where B is the colour
    // composited behind the current Gaussian (background first); with
    // B <- alpha c + (1 - alpha) B, S follows S <- S + alpha (G . c - S).
    float T[kPPT], G0[kPPT], G1[kPPT], G2[kPPT], S[kPPT];
    int32_t nc[kPPT];      // list positions below nc[j] were reached by pixel j (0 outside the image)
    float lsum = 0.0f;     // L1: this lane's sum of |image - target|
    // Every pixel's loads are issued unconditionally (pixels outside the image read
    // the nearest pixel inside, and their values are then replaced), so the four
    // pixels' loads are in flight together instead of one pixel after another.
#pragma unroll
    for (int j = 0; j < kPPT; j++) {
        const int64_t p = (int64_t)min(t.py[j], t.H - 1) * t.W + min(t.px[j], t.W - 1);
        const int64_t o = 3 * t.vbase + p;
        const bool in = t.inside[j];
        float gc[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            if (L1) {
                const float d = image[o + ch * HW] - target[o + ch * HW];
                lsum += in ? fabsf(d) : 0.0f;
                gc[ch] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
            } else {
                gc[ch] = dL_dimage[o + ch * HW];
            }
        }
        const float Tp = final_T[t.vbase + p];
        const int32_t np = n_contrib[t.vbase + p];
        G0[j] = in ? gc[0] : 0.0f;
        G1[j] = in ? gc[1] : 0.0f;
        G2[j] = in ? gc[2] : 0.0f;
        T[j] = in ? Tp : 1.0f;
        nc[j] = in ? np : 0;
    }
    if (L1) {
        // the tile's sum: DPP sums inside each row of 16 lanes, then the four row
        // totals added in FP64 in a fixed order
        float x = lsum;
        x += dpp<0xB1>(x);     // quad_perm [1,0,3,2]
        x += dpp<0x4E>(x);     // quad_perm [2,3,0,1]
        x += dpp<0x124>(x);    // row_ror:4
        x += dpp<0x128>(x);    // row_ror:8
        auto row = [&](int l) {
            return (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
        };
        const double tot = (row(0) + row(16)) + (row(32) + row(48));
        if (threadIdx.x == 0) tile_loss[t.tile] = tot;
    }
    const int2 rg = ranges[t.tile];
    const int32_t count = tile_entries[t.tile];
    const int64_t n_inst = *n_inst_dev;
    if (count == 0 || n_inst > cap) return;       // nothing composited here, or the sort overflowed
    const uint32_t gen = (uint32_t)n_inst_dev[1];  // this sort's generation: tags the slots written here
#pragma unroll
    for (int j = 0; j < kPPT; j++) S[j] = fmaf(G2[j], bg2, fmaf(G1[j], bg1, G0[j] * bg0));
    const int lane = threadIdx.x;
    int offA, offB;
    pair_offsets(lane, offA, offB);
    const uint32_t tag_bits = (lane == 8 || lane == 24) ? ~0u : 0u;   // lanes that store the generation tag
    // The (Gaussian, tile) sums go to the instance's own slot: no atomics, and the
    // projection adjoint adds a record's slots in a fixed order.  Raw buffer
    // stores over the slot's 40 bytes: the address stays scalar, and lanes whose
    // offset is 40 fall outside it and store nothing.
    auto store_pair = [&](float t, int32_t sa, int32_t sb) __attribute__((always_inline)) {
        const uint32_t w = (gen & tag_bits) | (__float_as_uint(t) & ~tag_bits);
        if (sa >= 0)
            __builtin_amdgcn_raw_buffer_store_b32(
                w, __builtin_amdgcn_make_buffer_rsrc(inst_grad + (int64_t)sa * kSlotWords, (short)0, 4 * kSlotWords, kBufWord3),
                offA, 0, 0);
        if (sb >= 0)
            __builtin_amdgcn_raw_buffer_store_b32(
                w, __builtin_amdgcn_make_buffer_rsrc(inst_grad + (int64_t)sb * kSlotWords, (short)0, 4 * kSlotWords, kBufWord3),
                offB, 0, 0);
    };
    // entries (composited Gaussians of this tile) back to front
    for (int32_t bend = count; bend > 0; bend -= BATCH) {
        const int32_t bstart = max(0, bend - BATCH);
        const int32_t cnt = bend - bstart;
        __syncthreads();
        for (int32_t i = lane; i < cnt; i += kLanes) {
            const uint32_t word = entries[rg.x + bstart + i];
            s_st[i].aux[1] = word;
            const int32_t gv = values[rg.x + (int32_t)(word >> 4)];
            const uint4 ts = reinterpret_cast<const uint4*>(tiles)[gv];     // the record's kept tiles
            const int32_t xlo = (int32_t)(ts.z & 0xffff), ylo = (int32_t)(ts.z >> 16);
            const int32_t w = (int32_t)(ts.w & 0xffff);
            const uint64_t mask = (uint64_t)ts.x | ((uint64_t)ts.y << 32);
            const int32_t slot = inst_first[gv] + kept_rank(mask, (t.ty - ylo) * w + (t.tx - xlo));
            const float lo = stage<TW, TH, false>(splats, gv, t.ox, t.oy, t.col0, t.row0, s_st, i);
            s_st[i].aux[0] = ((slot >= 0 && slot < n_inst) ? (uint32_t)slot : kNoSlot) | (may_clamp(lo) ? kSlotClamp : 0u);
        }
        __syncthreads();
        // one entry: its nine per-lane sums, as row sums and the ninth, and its slot
        auto entry = [&](const int32_t k, RowSums& rs, float& m8, int32_t& slot_out) __attribute__((always_inline)) {
            const float4 g = s_st[k].geo;
            const float4 cc = s_st[k].col;
            const float cb = s_st[k].blu;
            const float thr = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_st[k].thr)));
            const uint32_t word = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_st[k].aux[1]);
            const uint32_t sw = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_st[k].aux[0]);
            const int32_t slot = (sw & kNoSlot) == kNoSlot ? -1 : (int32_t)(sw & kNoSlot);
            const float lo = cc.y;    // a vector operand: the clamp flag comes with the slot
            const int32_t pos = (int32_t)(word >> 4);
            // Per-lane sums over the lane's pixels, later reduced over the wave:
            //   m[0..1] = sum dq' (dx, dy), m[2..4] = sum dq' (dx^2, dx dy, dy^2)
            //   with dq' = alpha dL/dalpha (so dL/dq = -dq'/2), m[5] = sum dq'
            //   (dL/do = m[5] / o, since alpha = o e^{-q/2} wherever dq' is not zero),
            //   m[6..8] = sum T alpha G (colour).
            // They start at -0, the additive identity, so the first block's adds fold away.
            float m[9];
#pragma unroll
            for (int i = 0; i < 9; i++) m[i] = -0.0f;
            // one block of the lane's four pixels (j and clamp are constants after inlining)
            auto block = [&](const int j, const bool clamp) __attribute__((always_inline)) {
                const float dx = t.fx[j] - g.x, dy = t.fy[j] - g.y;
                const float qs = quad(dx, dy, g.z, g.w, cc.x, lo);   // -q log2(e) / 2 + log2 o
                const float raw = raw_alpha(qs);
                const float al = clamp ? clamp_alpha(raw, kAlphaMax) : raw;   // the forward's alpha
                // the forward's decision: a pixel still compositing at this position took every
                // Gaussian inside the footprint with alpha >= 1/255 (it stops only after its last one)
                const bool in = pos < nc[j] && qs >= thr;
                const float ae = in ? al : 0.0f;      // 0 for pixels that did not take it: T, S unchanged
                const float Tk = T[j] * __builtin_amdgcn_rcpf(1.0f - ae);   // transmittance in front of k
                T[j] = Tk;
                const float w = Tk * ae;
                m[6] = fmaf(w, G0[j], m[6]);
                m[7] = fmaf(w, G1[j], m[7]);
                m[8] = fmaf(w, G2[j], m[8]);
                // G . (c - B) = G . c - S
                const float diff = fmaf(G2[j], cb, fmaf(G1[j], cc.w, fmaf(G0[j], cc.z, -S[j])));
                S[j] = fmaf(ae, diff, S[j]);
                // dq' = alpha dL/dalpha = T_k alpha G . (c - B): zero where the pixel did not take
                // the Gaussian (w = 0) and where the clamp holds alpha at 0.99
                float dqp = w * diff;
                if (clamp) dqp = al < kAlphaMax ? dqp : 0.0f;
                m[5] += dqp;
                const float px = dqp * dx;
                m[0] += px;
                m[1] = fmaf(dqp, dy, m[1]);
                m[2] = fmaf(px, dx, m[2]);
                m[3] = fmaf(px, dy, m[3]);
                m[4] = fmaf(dqp, dy * dy, m[4]);   // dy^2 is the quadratic's, shared by a row of blocks
            };
            // blocks whose bit is set, entered at the first one so that its code starts the
            // sums (a tile's entry always has at least one block)
            static_assert(kPPT == 4, "four blocks per tile");
            const uint32_t bits = word & ((1u << kPPT) - 1u);
            const int j0 = __builtin_ctz(bits);
            auto blocks = [&](const bool clamp) __attribute__((always_inline)) {
                if (j0 == 0) {
                    block(0, clamp);
                    if (bits & 2u) block(1, clamp);
                    if (bits & 4u) block(2, clamp);
                    if (bits & 8u) block(3, clamp);
                } else if (j0 == 1) {
                    block(1, clamp);
                    if (bits & 4u) block(2, clamp);
                    if (bits & 8u) block(3, clamp);
                } else if (j0 == 2) {
                    block(2, clamp);
                    if (bits & 8u) block(3, clamp);
                } else {
                    block(3, clamp);
                }
            };
            if (sw & kSlotClamp) blocks(true);
            else blocks(false);
            // the moments go to the slot as they are: the mean and conic gradients are
            // linear in them (dm = Q (m0, m1), d(a, b, c) = -(m2 / 2, m3, m4 / 2)), so the
            // projection adjoint forms them once per record from its summed slots
            rs = row_sums(m);
            m8 = m[8];
            slot_out = slot;
        };
        // entries in pairs, back to front (a staged batch is even except the tile's first)
        int32_t k = cnt - 1;
        for (; k >= 1; k -= 2) {
            RowSums ra, rb;
            float a8, b8;
            int32_t sa, sb;
            entry(k, ra, a8, sa);
            entry(k - 1, rb, b8, sb);
            store_pair(pair_totals(ra, a8, rb, b8, lane), sa, sb);
        }
        if (k == 0) {
            RowSums ra;
            float a8;
            int32_t sa;
            entry(0, ra, a8, sa);
            store_pair(pair_totals(ra, a8, RowSums{0.0f, 0.0f}, 0.0f, lane), sa, -1);
        }
    }
}

template <int TW, int TH, int BATCH>
void fwd_launch(const pg_views* v, const pg_splat* splats, const int32_t* values, const int32_t* ranges,
                const int32_t* order, const float bg[3], float* image, float* final_T, int32_t* n_contrib, int32_t* tile_entries,
                uint32_t* entries, uint64_t* counters, hipStream_t s) {
    const unsigned grid = (unsigned)v->n_tiles;
    if (counters)
        k_render_fwd<TW, TH, BATCH, true><<<grid, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), order, bg[0],
            bg[1], bg[2], image, final_T, n_contrib, tile_entries, entries,
            reinterpret_cast<unsigned long long*>(counters));
    else
        k_render_fwd<TW, TH, BATCH, false><<<grid, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, values, reinterpret_cast<const int2*>(ranges), order, bg[0],
            bg[1], bg[2], image, final_T, n_contrib, tile_entries, entries, nullptr);
}

template <int TW, int TH, int BATCH>
void bwd_launch(const pg_views* v, const pg_splat* splats, const pg_tile_set* tiles,
                const int32_t* values,
                const int32_t* ranges, const int32_t* order, const int32_t* inst_first, const int32_t* tile_entries,
                const uint32_t* entries, const int32_t* n_contrib, const float bg[3], const float* final_T,
                const float* dL_dimage, const int64_t* n_inst_dev, int64_t cap, float* inst_grad, const BwdL1* l1,
                hipStream_t s) {
    if (l1)
        k_render_bwd<TW, TH, BATCH, true><<<(unsigned)v->n_tiles, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, tiles, values, reinterpret_cast<const int2*>(ranges), order,
            inst_first, tile_entries, entries, n_contrib, bg[0], bg[1], bg[2], final_T, nullptr, n_inst_dev, cap,
            inst_grad, l1->image, l1->target, (float)(1.0 / (double)l1->n), l1->tile_loss);
    else
        k_render_bwd<TW, TH, BATCH, false><<<(unsigned)v->n_tiles, kLanes, 0, s>>>(
            v->d_views, v->n_views, v->n_tiles, splats, tiles, values, reinterpret_cast<const int2*>(ranges), order,
            inst_first, tile_entries, entries, n_contrib, bg[0], bg[1], bg[2], final_T, dL_dimage, n_inst_dev, cap,
            inst_grad, nullptr, nullptr, 0.0f, nullptr);
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
                             const int32_t* ranges, const int32_t* order, const float bg[3], float* image,
                             float* final_T, int32_t* n_contrib, int32_t* tile_entries, uint32_t* entries,
                             uint64_t* counters, hipStream_t s) {
    if (v->n_tiles == 0) return hipSuccess;
    dispatch<FwdRun>(v->tiling, v, splats, values, ranges, order, bg, image, final_T, n_contrib, tile_entries, entries,
                     counters, s);
    return hipGetLastError();
}

hipError_t launch_render_bwd(const pg_views* v, const pg_splat* splats, const pg_tile_set* tiles, const int32_t* values,
                             const int32_t* ranges, const int32_t* order, const int32_t* inst_first,
                             const int32_t* tile_entries, const uint32_t* entries, const int32_t* n_contrib,
                             const float bg[3], const float* final_T, const float* dL_dimage,
                             const int64_t* n_inst_dev, int64_t cap, float* inst_grad, const BwdL1* l1,
                             hipStream_t s) {
    if (v->n_tiles == 0) return hipSuccess;
    dispatch<BwdRun>(v->tiling, v, splats, tiles, values, ranges, order, inst_first, tile_entries, entries, n_contrib, bg,
                     final_T, dL_dimage, n_inst_dev, cap, inst_grad, l1, s);
    return hipGetLastError();
}

}  // namespace pg
