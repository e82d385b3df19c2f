// a3 -- tile binning and depth sort.
//
// Every projected Gaussian is listed once per screen tile its rectangle
// covers (the 3DGS tile rasteriser the paper names, Sec. 3), keyed by
// (global tile << 32 | fp32 depth bits), and the instances are sorted by that
// key so each tile's list is front to back (depth sort per camera,
// supplementary viewer section).  Because the instances are emitted in
// ascending gv order and the sort is a stable LSD radix sort, equal depths
// stay in ascending Gaussian id order.
//
// Kernels (all HBM-bound):
//   k_bin_count     per 1024 (view, Gaussian) records: sum of tiles touched
//   scan            exclusive scan of the block sums -> instance offsets
//   k_emit          work-group-cooperative emission: the group's output range
//                   is written contiguously (coalesced), each lane locating its
//                   (record, tile) by binary search over the group's prefix sums
//   radix passes    per 8-bit digit: upsweep histogram, scan, downsweep
//                   (wave-level multisplit ranking with ballots, LDS staging so
//                   the scatter writes digit runs contiguously)
//   k_ranges        [start, end) of every tile from the sorted keys
// Counts that only the device knows (instances) are read from device memory,
// so the chain needs no host synchronisation.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kEmitThreads = 1024;
constexpr int kSortGrid = 2048;      // persistent grid of the radix kernels (grid-stride over tiles)

struct SortWs {
    int64_t* block_sums;
    int64_t* block_offs;
    int64_t* scan_tmp;
    int64_t* misc;          // [0] instances to sort (0 on overflow), [1] 256 * sort tiles
    uint64_t* keys_alt;
    int32_t* vals_alt;
    int32_t* counts;
    int32_t* count_offs;
};

int64_t n_emit_blocks(const pg_views* v) { return ceil_div(v->n_gv, kEmitThreads); }

SortWs carve(const pg_views* v, int64_t cap, void* ws, size_t* total) {
    SortWs w{};
    const int64_t nb = imax(n_emit_blocks(v), 1);
    const int64_t ntile = imax(ceil_div(cap, kSortTile), 1);
    char* p = (char*)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = p + off;
        off += align256(bytes);
        return q;
    };
    w.block_sums = (int64_t*)take(nb * 8);
    w.block_offs = (int64_t*)take(nb * 8);
    w.scan_tmp = (int64_t*)take(kScanTmpWords * 8);
    w.misc = (int64_t*)take(4 * 8);
    w.keys_alt = (uint64_t*)take(imax(cap, 1) * 8);
    w.vals_alt = (int32_t*)take(imax(cap, 1) * 4);
    w.counts = (int32_t*)take(ntile * kRadix * 4);
    w.count_offs = (int32_t*)take(ntile * kRadix * 4);
    if (total) *total = off;
    return w;
}

__global__ __launch_bounds__(kEmitThreads) void k_bin_count(const pg_bin* __restrict__ bins, int64_t n_gv,
                                                            int64_t* __restrict__ block_sums) {
    __shared__ int64_t s[kEmitThreads / 64];
    const int64_t gv = (int64_t)blockIdx.x * kEmitThreads + threadIdx.x;
    int64_t c = gv < n_gv ? (int64_t)bins[gv].n_tiles : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < kEmitThreads / 64; k++) t += s[k];
        block_sums[blockIdx.x] = t;
    }
}

__global__ void k_post_count(const int64_t* n_inst, int64_t cap, int32_t* overflow, int64_t* misc) {
    const int64_t I = *n_inst;
    const bool of = I > cap;
    *overflow = of ? 1 : 0;
    const int64_t eff = of ? 0 : I;
    misc[0] = eff;
    misc[1] = ceil_div(eff, kSortTile) * kRadix;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit(const pg_bin* __restrict__ bins, int64_t n_gv, int64_t N,
                                                       const ViewDev* __restrict__ views,
                                                       const int64_t* __restrict__ block_offs,
                                                       const int64_t* __restrict__ misc, uint64_t* __restrict__ keys,
                                                       int32_t* __restrict__ vals) {
    __shared__ int32_t s_incl[kEmitThreads];
    __shared__ uint2 s_rect[kEmitThreads];
    __shared__ uint32_t s_key[kEmitThreads];
    __shared__ int32_t s_warp[kEmitThreads / 64];
    if (misc[0] == 0) return;   // overflow (or nothing to emit): uniform exit
    const int t = threadIdx.x;
    const int64_t gv0 = (int64_t)blockIdx.x * kEmitThreads;
    const int64_t gv = gv0 + t;
    int32_t nt = 0;
    if (gv < n_gv) {
        const uint4 b = reinterpret_cast<const uint4*>(bins)[gv];
        nt = (int32_t)b.w;
        s_rect[t] = make_uint2(b.x, b.y);
        s_key[t] = b.z;
    }
    const int lane = t & 63, wid = t >> 6;
    int32_t v = nt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_warp[wid] = v;
    __syncthreads();
    int32_t before = 0;
    for (int k = 0; k < wid; k++) before += s_warp[k];
    s_incl[t] = v + before;
    __syncthreads();
    const int32_t total = s_incl[kEmitThreads - 1];
    const int64_t base = block_offs[blockIdx.x];
    for (int32_t p = t; p < total; p += kEmitThreads) {
        int lo = 0, hi = kEmitThreads - 1;     // first j with s_incl[j] > p
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_incl[mid] > p) hi = mid; else lo = mid + 1;
        }
        const int32_t k = p - (lo ? s_incl[lo - 1] : 0);
        const uint2 r = s_rect[lo];
        const int32_t xlo = (int32_t)(r.x & 0xffff), ylo = (int32_t)(r.x >> 16);
        const int32_t xhi = (int32_t)(r.y & 0xffff);
        const int32_t w = xhi - xlo + 1;
        const int32_t tx = xlo + k % w, ty = ylo + k / w;
        const int64_t g = gv0 + lo;
        const int64_t view = g / N;
        const ViewDev& V = views[view];
        const uint64_t tile = (uint64_t)(V.tile_base + (int64_t)ty * V.TX + tx);
        keys[base + p] = (tile << 32) | (uint64_t)s_key[lo];
        vals[base + p] = (int32_t)g;
    }
}

// Peers of this lane: active lanes holding the same 8-bit digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool active) {
    uint64_t peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < kRadixBits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_upsweep(const uint64_t* __restrict__ keys,
                                                                const int64_t* __restrict__ misc, int shift,
                                                                int32_t* __restrict__ counts) {
    __shared__ uint32_t s_cnt[kRadix];
    const int64_t I = misc[0];
    const int64_t ntile = ceil_div(I, kSortTile);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t b = blockIdx.x; b < ntile; b += gridDim.x) {
        s_cnt[threadIdx.x] = 0;
        __syncthreads();
        const int64_t start = b * kSortTile + (int64_t)wid * (kSortTile / 4);
#pragma unroll 4
        for (int r = 0; r < kSortItems; r++) {
            const int64_t idx = start + r * 64 + lane;
            const bool active = idx < I;
            const uint32_t d = active ? (uint32_t)((keys[idx] >> shift) & (kRadix - 1)) : 0u;
            const uint64_t peers = match_digit(d, active);
            const uint64_t below = peers & ((1ull << lane) - 1ull);
            if (active && below == 0) atomicAdd(&s_cnt[d], (uint32_t)__popcll(peers));
        }
        __syncthreads();
        counts[(int64_t)threadIdx.x * ntile + b] = (int32_t)s_cnt[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_radix_downsweep(const uint64_t* __restrict__ keys_in,
                                                                  const int32_t* __restrict__ vals_in,
                                                                  uint64_t* __restrict__ keys_out,
                                                                  int32_t* __restrict__ vals_out,
                                                                  const int64_t* __restrict__ misc, int shift,
                                                                  const int32_t* __restrict__ count_offs) {
    __shared__ uint32_t s_hist[4][kRadix];
    __shared__ uint32_t s_boff[kRadix];
    __shared__ int32_t s_glob[kRadix];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_keys[kSortTile];
    __shared__ int32_t s_vals[kSortTile];
    const int64_t I = misc[0];
    const int64_t ntile = ceil_div(I, kSortTile);
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    for (int64_t b = blockIdx.x; b < ntile; b += gridDim.x) {
        for (int w = 0; w < 4; w++) s_hist[w][t] = 0;
        __syncthreads();
        const int64_t start = b * kSortTile + (int64_t)wid * (kSortTile / 4);
        uint64_t key[kSortItems];
        int32_t val[kSortItems];
        uint32_t rank[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; r++) {
            const int64_t idx = start + r * 64 + lane;
            const bool active = idx < I;
            key[r] = active ? keys_in[idx] : 0ull;
            val[r] = active ? vals_in[idx] : 0;
            const uint32_t d = (uint32_t)((key[r] >> shift) & (kRadix - 1));
            const uint64_t peers = match_digit(d, active);
            const uint64_t below = peers & ((1ull << lane) - 1ull);
            const uint32_t base = s_hist[wid][d];
            rank[r] = base + (uint32_t)__popcll(below);
            if (active && below == 0) s_hist[wid][d] = base + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit: exclusive over waves, then exclusive over digits of the block totals
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            const uint32_t c = s_hist[w][t];
            s_hist[w][t] = run;
            run += c;
        }
        s_glob[t] = count_offs[(int64_t)t * ntile + b];
        uint32_t incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_wsum[wid] = incl;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wid; w++) pre += s_wsum[w];
        s_boff[t] = pre + incl - run;
        __syncthreads();
        const int64_t tile_n = imin(kSortTile, I - b * kSortTile);
#pragma unroll
        for (int r = 0; r < kSortItems; r++) {
            const int64_t idx = start + r * 64 + lane;
            if (idx < I) {
                const uint32_t d = (uint32_t)((key[r] >> shift) & (kRadix - 1));
                const uint32_t pos = s_boff[d] + s_hist[wid][d] + rank[r];
                s_keys[pos] = key[r];
                s_vals[pos] = val[r];
            }
        }
        __syncthreads();
        for (int64_t i = t; i < tile_n; i += kSortThreads) {
            const uint64_t k = s_keys[i];
            const uint32_t d = (uint32_t)((k >> shift) & (kRadix - 1));
            const int64_t o = (int64_t)s_glob[d] + (i - (int64_t)s_boff[d]);
            keys_out[o] = k;
            vals_out[o] = s_vals[i];
        }
        __syncthreads();
    }
}

__global__ void k_ranges(const uint64_t* __restrict__ keys, const int64_t* __restrict__ misc,
                         int32_t* __restrict__ ranges) {
    const int64_t I = misc[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t tile = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[2 * (int64_t)tile] = (int32_t)i;
        if (i == I - 1 || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[2 * (int64_t)tile + 1] = (int32_t)(i + 1);
    }
}

}  // namespace

size_t sort_ws_bytes(const pg_views* v, int64_t cap) {
    size_t total = 0;
    carve(v, cap, nullptr, &total);
    return total;
}

hipError_t launch_bin_sort(const pg_views* v, const pg_bin* bins, int64_t cap, uint64_t* keys, int32_t* values,
                           int32_t* ranges, int64_t* n_inst_dev, int32_t* overflow_dev, void* ws, hipStream_t s) {
    SortWs w = carve(v, cap, ws, nullptr);
    const int64_t nb = n_emit_blocks(v);
    hipError_t e = fill_u32(ranges, 0u, 2 * v->n_tiles, s);
    if (e != hipSuccess) return e;
    if (nb > 0) {
        k_bin_count<<<(unsigned)nb, kEmitThreads, 0, s>>>(bins, v->n_gv, w.block_sums);
        e = scan_i64(w.block_sums, w.block_offs, nullptr, 0, nb, n_inst_dev, w.scan_tmp, s);
        if (e != hipSuccess) return e;
    } else {
        e = fill_u32(n_inst_dev, 0u, 2, s);
        if (e != hipSuccess) return e;
    }
    k_post_count<<<1, 1, 0, s>>>(n_inst_dev, cap, overflow_dev, w.misc);
    const int passes = v->sort_passes;
    // emit into the buffer that makes the last pass land in the caller's arrays
    uint64_t* kA = (passes % 2 == 0) ? keys : w.keys_alt;
    int32_t* vA = (passes % 2 == 0) ? values : w.vals_alt;
    uint64_t* kB = (passes % 2 == 0) ? w.keys_alt : keys;
    int32_t* vB = (passes % 2 == 0) ? w.vals_alt : values;
    if (nb > 0)
        k_emit<<<(unsigned)nb, kEmitThreads, 0, s>>>(bins, v->n_gv, v->n_gauss, v->d_views, w.block_offs, w.misc, kA,
                                                     vA);
    const unsigned grid = (unsigned)imax(1, imin(kSortGrid, ceil_div(cap, kSortTile)));
    for (int p = 0; p < passes; p++) {
        const int shift = p * kRadixBits;
        k_radix_upsweep<<<grid, kSortThreads, 0, s>>>(kA, w.misc, shift, w.counts);
        e = scan_i32(w.counts, w.count_offs, w.misc + 1, 1, 0, nullptr, w.scan_tmp, s);
        if (e != hipSuccess) return e;
        k_radix_downsweep<<<grid, kSortThreads, 0, s>>>(kA, vA, kB, vB, w.misc, shift, w.count_offs);
        uint64_t* tk = kA; kA = kB; kB = tk;
        int32_t* tv = vA; vA = vB; vB = tv;
    }
    k_ranges<<<1024, 256, 0, s>>>(keys, w.misc, ranges);
    return hipGetLastError();
}

}  // namespace pg
