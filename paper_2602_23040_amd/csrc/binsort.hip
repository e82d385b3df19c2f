// a3 -- tile binning and depth sort.
//
// Every projected Gaussian is listed once per kept screen tile of its
// rectangle (the 3DGS tile rasteriser the paper names, Sec. 3; the projection
// drops tiles the ellipse q <= 9 cannot reach), and each tile's
// list is ordered front to back by camera-space depth (depth sort per camera,
// supplementary viewer section), equal depths by ascending Gaussian id.
//
// The order is built in two stable radix sorts instead of one sort of
// (tile, depth) keys over all instances:
//   1. the surviving (view, Gaussian) records -- far fewer than instances --
//      are compacted in (view, id) order and stably sorted by their fp32
//      depth bits alone (all views mixed);
//   2. instances are emitted in that order (each record lists the kept tiles
//      of its rectangle) and stably sorted by global tile id alone.
// Because the second sort is stable and every tile belongs to one view, each
// tile's list comes out ordered by (depth, id): equal depths keep the
// compaction order, which inside one view is ascending id.  That is the order
// of sorting (tile, depth, id) keys, with 32-bit keys in both sorts.
//
// Kernels (all HBM-bound):
//   k_valid_count / k_compact   records with n_tiles > 0 -> (depth bits, gv);
//                               inst_first[gv] = instances of all records before
//                               gv in (view, id) order: the record's gradient
//                               slots, one per kept tile in rectangle order
//   radix passes (32-bit keys)  LSD, four 8-bit digits of the depth bits
//   k_sorted_count / k_emit     tiles per sorted record -> instance offsets ->
//                               work-group-cooperative emission (coalesced writes)
//   radix passes (32-bit keys)  tile ids, 6-bit digits
//   k_ranges                    [start, end) of every tile
//   k_order_count/_scan/_place  the compositing kernels' tile dispatch order
// Radix passes: one histogram kernel counts every digit of the sort in one
// read of the keys; then one kernel per digit ranks each 4096-key tile with a
// wave-level multisplit (one ballot per digit bit), takes each digit's output
// offset from the counts of the tiles before it (decoupled look-back), and
// scatters through LDS so each digit's run is written contiguously.  Counts
// that only the device knows are read from device memory, so the chain needs
// no host synchronisation.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kBlk = 1024;           // records per compaction / emission work-group

struct DigitPlan {
    int passes, digit;      // LSD passes of equal width digit bits
};
constexpr int kOsMaxBits = 9;                // digit width the radix pass kernels are built for
constexpr int kDepthDigitBits = 8;           // digit width caps of the record (depth) and instance (tile) sorts
constexpr int kTileDigitBits = 7;            // 18-bit tile ids: 3 x 6 bits; 19-21 bits: 3 x 7 instead of 4 x 5

DigitPlan digit_plan(int bits, int max_bits) {
    DigitPlan p;
    p.passes = (int)imax((bits + max_bits - 1) / max_bits, 1);
    p.digit = (bits + p.passes - 1) / p.passes;
    return p;
}

struct SortPlan {
    DigitPlan depth, tile;  // record sort (32-bit depth keys), instance sort (tile ids)
};

SortPlan plan_for(const pg_views* v) {
    SortPlan p;
    p.depth = digit_plan(32, kDepthDigitBits);
    p.tile = digit_plan(v->key_bits, kTileDigitBits);   // ceil(log2(n_tiles)), >= 1
    return p;
}

size_t os_ws_bytes(int64_t cap, DigitPlan pl);

struct SortWs {
    int64_t* blk_a;          // per-block sums (compaction / emission)
    int64_t* blk_a_off;
    int64_t* blk_b;          // per-block tile sums in (view, id) order (slot offsets)
    int64_t* blk_b_off;
    int64_t* scan_tmp;
    int64_t* misc;           // [0] valid records, [1] instances to sort (0 on overflow), [4] instances (slot scan)
    uint32_t* rk0;           // record sort ping-pong
    uint32_t* rk1;
    int32_t* rv0;
    int32_t* rv1;
    uint4* stiles;           // the records' tile sets gathered in depth order (read by the emission)
    uint32_t* tk_alt;        // tile sort ping-pong partner of the caller's arrays
    int32_t* tv_alt;
    char* os;                // radix pass state (histograms, look-back status), shared by both sorts
    int32_t* order_cnt;      // tile dispatch order: per (tile group, length class) counts
    int32_t* order_base;     // ... and their class-major exclusive scan
    int32_t* order_cls;      // ... first slot and size of each class
};

int64_t n_blocks(const pg_views* v) { return imax(ceil_div(v->n_gv, kBlk), 1); }

constexpr int kOrderClasses = 64; // length classes of the tile dispatch order (four per octave)
constexpr int kOrderBlk = 256;

SortWs carve(const pg_views* v, int64_t cap, void* ws, size_t* total) {
    const SortPlan pl = plan_for(v);
    SortWs w{};
    const int64_t nb = n_blocks(v);
    const int64_t ngv = imax(v->n_gv, 1);
    char* p = (char*)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = p + off;
        off += align256(bytes);
        return q;
    };
    w.blk_a = (int64_t*)take(nb * 8);
    w.blk_a_off = (int64_t*)take(nb * 8);
    w.blk_b = (int64_t*)take(nb * 8);
    w.blk_b_off = (int64_t*)take(nb * 8);
    w.scan_tmp = (int64_t*)take(kScanTmpWords * 8);
    w.misc = (int64_t*)take(8 * 8);
    w.rk0 = (uint32_t*)take(ngv * 4);
    w.rk1 = (uint32_t*)take(ngv * 4);
    w.rv0 = (int32_t*)take(ngv * 4);
    w.rv1 = (int32_t*)take(ngv * 4);
    w.stiles = (uint4*)take(ngv * 16);
    w.tk_alt = (uint32_t*)take(imax(cap, 1) * 4);
    w.tv_alt = (int32_t*)take(imax(cap, 1) * 4);
    w.os = take(std::max(os_ws_bytes(ngv, pl.depth), os_ws_bytes(cap, pl.tile)));
    const int64_t order_words = ceil_div(imax(v->n_tiles, 1), kOrderBlk) * kOrderClasses;
    w.order_cnt = (int32_t*)take(order_words * 4);
    w.order_base = (int32_t*)take(order_words * 4);
    w.order_cls = (int32_t*)take(2 * kOrderClasses * 4);
    if (total) *total = off;
    return w;
}

// Inclusive scan of one int per thread over a kBlk work-group.
__device__ __forceinline__ int32_t block_incl_1024(int32_t v, int32_t* s_warp) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_warp[wid] = v;
    __syncthreads();
    int32_t before = 0;
    for (int k = 0; k < wid; k++) before += s_warp[k];
    return v + before;
}

__device__ __forceinline__ int64_t block_incl_1024_i64(int64_t v, int64_t* s_warp) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_warp[wid] = v;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < wid; k++) before += s_warp[k];
    return v + before;
}

__device__ __forceinline__ int64_t block_sum_1024(int64_t c, int64_t* s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < kBlk / 64; k++) t += s[k];
    return t;
}

__global__ __launch_bounds__(kBlk) void k_valid_count(const pg_bin* __restrict__ bins, int64_t n_gv,
                                                      int64_t* __restrict__ blk_cnt, int64_t* __restrict__ blk_nt) {
    __shared__ int64_t s[kBlk / 64];
    const int64_t gv = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int64_t nt = gv < n_gv ? (int64_t)bins[gv].n_tiles : 0;
    const int64_t c = block_sum_1024(nt > 0 ? 1 : 0, s);
    __syncthreads();
    const int64_t t = block_sum_1024(nt, s);
    if (threadIdx.x == 0) {
        blk_cnt[blockIdx.x] = c;
        blk_nt[blockIdx.x] = t;
    }
}

// Compaction of the surviving records (key: depth bits, value: gv) and the
// instance-slot offsets in (view, id) order: inst_first[gv] = number of
// instances of all records before gv.
__global__ __launch_bounds__(kBlk) void k_compact(const pg_bin* __restrict__ bins, int64_t n_gv,
                                                  const int64_t* __restrict__ blk_off,
                                                  const int64_t* __restrict__ blk_nt_off, uint32_t* __restrict__ rk,
                                                  int32_t* __restrict__ rv, int32_t* __restrict__ inst_first) {
    __shared__ int32_t s_warp[kBlk / 64];
    __shared__ int64_t s_warp64[kBlk / 64];
    const int64_t gv = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    uint4 b = make_uint4(0u, 0u, 0u, 0u);
    if (gv < n_gv) b = reinterpret_cast<const uint4*>(bins)[gv];
    const int32_t valid = (gv < n_gv && b.w > 0) ? 1 : 0;
    const int32_t incl = block_incl_1024(valid, s_warp);
    const int64_t nt = valid ? (int64_t)b.w : 0;
    const int64_t nt_incl = block_incl_1024_i64(nt, s_warp64);
    if (gv < n_gv) inst_first[gv] = (int32_t)(blk_nt_off[blockIdx.x] + nt_incl - nt);
    if (valid) {
        const int64_t pos = blk_off[blockIdx.x] + incl - 1;
        rk[pos] = b.z;
        rv[pos] = (int32_t)gv;
    }
}

// Tile sets gathered into depth order (one 16-byte read per record) and the
// group sums of the kept-tile counts.
// The sorted records are in rv_moved, or in rv_stayed when the depth sort's
// last pass had one digit for every key and moved nothing (*stayed).
__global__ __launch_bounds__(kBlk) void k_sorted_count(const pg_tile_set* __restrict__ tiles,
                                                       const int32_t* __restrict__ rv_moved,
                                                       const int32_t* __restrict__ rv_stayed,
                                                       const uint32_t* __restrict__ stayed,
                                                       const int64_t* __restrict__ misc, int64_t* __restrict__ blk,
                                                       uint4* __restrict__ stiles) {
    __shared__ int64_t s[kBlk / 64];
    const int32_t* __restrict__ rv = *stayed ? rv_stayed : rv_moved;
    const int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    int64_t c = 0;
    if (p < misc[0]) {
        const uint4 ts = reinterpret_cast<const uint4*>(tiles)[rv[p]];
        stiles[p] = ts;
        c = (int64_t)kept_count(ts);
    }
    const int64_t t = block_sum_1024(c, s);
    if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

// Overflow check and the next sort generation (n_inst[1], never 0: slots the
// adjoint has not written this generation, zero-filled ones included, read
// as zero).
__global__ void k_post_count(int64_t* n_inst, int64_t cap, int32_t* overflow, int64_t* misc) {
    uint32_t gen = (uint32_t)n_inst[1] + 1u;
    n_inst[1] = (int64_t)(gen == 0u ? 1u : gen);
    const int64_t I = *n_inst;
    const bool of = I > cap;
    *overflow = (*overflow & 2) | (of ? 1 : 0);
    const int64_t eff = of ? 0 : I;
    misc[1] = eff;
}


// Emission in sorted-record order.  The group's 1024 records own consecutive
// output ranges (their kept-tile counts scanned over the group); each thread
// walks its own record's kept-tile bits in increasing order (row-major over
// the rectangle) and writes (tile, gv) at its range, so an instance costs a
// bit scan and one small division.  The lanes of a wave write into one
// window of the output a few hundred instances long.  Records keeping every
// tile of a rectangle larger than 64 tiles are rare and long: their waves
// emit them one after another, all 64 lanes on one record.
__device__ __forceinline__ void rect_tile(int32_t k, int32_t w, float rw, int32_t& row, int32_t& col) {
    // row = k / w from a float estimate (k < 2^24), corrected to the exact quotient
    row = (int32_t)((float)k * rw);
    col = k - row * w;
    if (col < 0) { row--; col += w; }
    else if (col >= w) { row++; col -= w; }
}

__global__ __launch_bounds__(kBlk) void k_emit(const uint4* __restrict__ stiles, const int32_t* __restrict__ rv_moved,
                                               const int32_t* __restrict__ rv_stayed,
                                               const uint32_t* __restrict__ stayed, int64_t N,
                                               const ViewDev* __restrict__ views,
                                               const int64_t* __restrict__ blk_off, const int64_t* __restrict__ misc,
                                               uint32_t* __restrict__ tkeys, int32_t* __restrict__ tvals) {
    const int32_t* __restrict__ rv = *stayed ? rv_stayed : rv_moved;   // as in k_sorted_count
    __shared__ int32_t s_warp[kBlk / 64];
    if (misc[1] == 0) return;   // overflow (or nothing to emit): uniform exit
    const int t = threadIdx.x, lane = t & 63;
    const int64_t p = (int64_t)blockIdx.x * kBlk + t;
    int32_t nt = 0, gv = 0, w = 1, tx = 0;
    uint32_t tile0 = 0u;
    uint64_t mask = 0;
    if (p < misc[0]) {
        gv = rv[p];
        const uint4 ts = stiles[p];
        nt = kept_count(ts);
        const int32_t xlo = (int32_t)(ts.z & 0xffff), ylo = (int32_t)(ts.z >> 16);
        const ViewDev& V = views[gv / N];
        w = (int32_t)(ts.w & 0xffff);
        tx = V.TX;
        tile0 = (uint32_t)(V.tile_base + (int64_t)ylo * V.TX + xlo);
        mask = (uint64_t)ts.x | ((uint64_t)ts.y << 32);
    }
    const int32_t incl = block_incl_1024(nt, s_warp);
    const int64_t e0 = blk_off[blockIdx.x] + incl - nt;     // this record's first output
    const float rw = 1.0f / (float)w;
    if (mask != 0) {
        uint64_t m = mask;
        for (int64_t e = e0; m != 0; e++) {
            const int32_t bit = (int32_t)__builtin_ctzll(m);
            m &= m - 1;
            int32_t row, col;
            rect_tile(bit, w, rw, row, col);
            tkeys[e] = tile0 + (uint32_t)(row * tx + col);
            tvals[e] = gv;
        }
    }
    // records that keep every tile of their rectangle, one at a time per wave
    uint64_t big = __ballot(mask == 0 && nt > 0);
    while (big) {
        const int src = __builtin_ctzll(big);
        big &= big - 1;
        const int32_t bn = __shfl(nt, src, 64), bw = __shfl(w, src, 64), btx = __shfl(tx, src, 64);
        const int32_t bgv = __shfl(gv, src, 64);
        const uint32_t bt0 = (uint32_t)__shfl((int)tile0, src, 64);
        const int64_t be0 = __shfl(e0, src, 64);
        const float brw = 1.0f / (float)bw;
        for (int32_t k = lane; k < bn; k += 64) {
            int32_t row, col;
            rect_tile(k, bw, brw, row, col);
            tkeys[be0 + k] = bt0 + (uint32_t)(row * btx + col);
            tvals[be0 + k] = bgv;
        }
    }
}

// Peers of this lane: active lanes holding the same BITS-bit digit.  Per
// bit, the ballot of the lanes that have it set, flipped where this lane's
// bit is clear, marks the lanes that differ from it in that bit; a peer
// differs in none.  Each half of the 64-lane mask costs an exclusive-or with
// the lane's sign-extended bit and an or per bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool active) {
    uint32_t diff_lo = 0u, diff_hi = 0u;
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);   // all ones where this lane's bit is set
        const uint64_t m = __ballot(s != 0u);
        diff_lo |= (uint32_t)m ^ s;
        diff_hi |= (uint32_t)(m >> 32) ^ s;
    }
    const uint64_t eq = ~(((uint64_t)diff_hi << 32) | diff_lo);
    return eq & __ballot(active);
}

// ------------------------------------------------------------------ onesweep LSD radix passes
// One kernel per digit.  Work-group b ranks the keys of radix tile b (4096
// pairs) with the wave multisplit, publishes its digit counts, and finds
// each digit's output offset by looking back over the tiles before it
// (decoupled look-back): a tile's status word per digit holds either its own
// count (AGG) or the count of that digit over every tile up to and including
// it (PRE).  The digit offsets over the whole input come from one histogram
// pass over the keys for every digit of the sort.  A pass reads and writes
// each pair once.
// Waiting on lower-numbered work-groups cannot deadlock because every XCD
// starts its share of the grid in index order: the lowest-numbered unfinished
// work-group has no unfinished predecessor, and if it had not started, its
// XCD would hold only finished lower-numbered groups and so have room for it.
// (An atomic ticket per work-group, which does not rely on that order, made
// the passes 15 % slower.)  The wait is bounded anyway: a look-back that
// polls kLookbackSpins times gives up, and the sort reports it.
constexpr uint32_t kStAgg = 1u, kStPre = 2u;
constexpr int kLookbackSpins = 1 << 22;      // a bound that a working chain never reaches (~1 s of polling)
constexpr int kMaxSortPasses = 4;
constexpr int kLookWindow = 8;               // predecessors read at once by the look-back

__device__ __forceinline__ void st_publish(unsigned long long* p, uint32_t flag, uint32_t value) {
    __hip_atomic_store(p, ((unsigned long long)flag << 32) | value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long st_read(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back: the sum of the values of work-groups 0 .. b-1 (b > 0)
// from their status words (work-group k's at p[k * stride]), read
// kLookWindow at a time from b - 1 backwards (a first wave of work-groups
// starts together, and one dependent load per predecessor would make its
// walks long) and added until a word flagged kStPre (an inclusive prefix).  A
// word not yet published is read again; after kLookbackSpins waits the walk
// gives up and sets *err (never in a working chain: report, do not hang).
__device__ __forceinline__ uint32_t lookback_excl(unsigned long long* p, int64_t stride, int64_t b, int32_t* err) {
    uint32_t excl = 0;
    int64_t k = b - 1;          // newest predecessor not yet added
    int spins = 0;
    bool done = false;
    while (!done) {
        unsigned long long w[kLookWindow];
#pragma unroll
        for (int j = 0; j < kLookWindow; j++) w[j] = k - j >= 0 ? st_read(&p[(k - j) * stride]) : 0ull;
        // newest first: add counts until a PRE word; stop at a word not published yet
        int adv = 0;
        bool stop = false;
#pragma unroll
        for (int j = 0; j < kLookWindow; j++) {
            const uint32_t flag = (uint32_t)(w[j] >> 32);
            if (!stop && !done) {
                if (k - j < 0 || flag == 0u) {
                    stop = true;
                } else {
                    excl += (uint32_t)w[j];
                    adv = j + 1;
                    done = flag == kStPre || k - j == 0;
                }
            }
        }
        if (done) break;
        k -= adv;
        if (adv < kLookWindow) {      // waiting on an unpublished word
            if (++spins > kLookbackSpins) {
                atomicOr(err, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// Digit counts of every pass of a sort in one read of the keys:
// hist[p NB + d] = keys whose bits [p BITS, (p + 1) BITS) equal d.  Each wave
// counts into its own LDS histogram; with UNIFORM, a wave whose active lanes
// share a digit adds once (depth keys share their high bits, which would
// otherwise serialise the LDS atomics).
template <int BITS, bool UNIFORM>
__global__ __launch_bounds__(256) void k_os_hist(const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_ptr,
                                                 int passes, uint32_t* __restrict__ hist) {
    constexpr int NB = 1 << BITS;
    constexpr int KPT = 16;                      // keys per thread per sweep, all loaded before they are counted
    __shared__ uint32_t s[4][kMaxSortPasses * NB];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < passes * NB; i += 256) {
#pragma unroll
        for (int w = 0; w < 4; w++) s[w][i] = 0;
    }
    __syncthreads();
    const int64_t n = *n_ptr;
    uint32_t* sw = s[wid];
    for (int64_t base = (int64_t)blockIdx.x * 256 * KPT; base < n; base += (int64_t)gridDim.x * 256 * KPT) {
        uint32_t k[KPT];
#pragma unroll
        for (int j = 0; j < KPT; j++) {
            const int64_t i = base + (int64_t)j * 256 + threadIdx.x;
            k[j] = i < n ? keys[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < KPT; j++) {
            const bool active = base + (int64_t)j * 256 + threadIdx.x < n;
            if (!UNIFORM) {
                if (active)
                    for (int p = 0; p < passes; p++) atomicAdd(&sw[p * NB + ((k[j] >> (p * BITS)) & (NB - 1))], 1u);
                continue;
            }
            const uint64_t act = __ballot(active);
            if (act == 0) break;
            const int lead = __builtin_ctzll(act);
            for (int p = 0; p < passes; p++) {
                const uint32_t d = (k[j] >> (p * BITS)) & (NB - 1);
                const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, lead);
                if (__ballot(active && d == d0) == act) {
                    if (lane == lead) atomicAdd(&sw[p * NB + d0], (uint32_t)__popcll(act));   // counts only: order-free
                } else if (active) {
                    atomicAdd(&sw[p * NB + d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * NB; i += 256) {
        const uint32_t c = s[0][i] + s[1][i] + s[2][i] + s[3][i];
        if (c) atomicAdd(&hist[i], c);
    }
}

// Exclusive scan of each pass's digit counts (one work-group of 512 threads);
// uni[p] = 1 when one digit of pass p holds every key (the pass is then the
// identity permutation).
__global__ __launch_bounds__(512) void k_os_scan(uint32_t* __restrict__ hist, int passes, int nb,
                                                 const int64_t* __restrict__ n_ptr, uint32_t* __restrict__ uni) {
    __shared__ uint32_t s_w[8];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int64_t n = *n_ptr;
    for (int p = 0; p < passes; p++) {
        const uint32_t c = t < nb ? hist[p * nb + t] : 0u;
        const int all_one = __syncthreads_or(n > 0 && (int64_t)c == n);
        if (t == 0) uni[p] = (uint32_t)all_one;
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wid; w++) before += s_w[w];
        if (t < nb) hist[p * nb + t] = before + incl - c;
        __syncthreads();
    }
}

// Clears what the passes of one sort count on: the histograms, the look-back
// error flag and the status words of the tiles the device-side
// count needs (status is [pass][tile][NB], tile stride NB, pass stride
// tiles_max NB).
__global__ void k_os_clear(const int64_t* __restrict__ n_ptr, int passes, int nb, int64_t tiles_max,
                           unsigned long long* __restrict__ status, uint32_t* __restrict__ hist,
                           int32_t* __restrict__ err) {
    const int64_t ntile = imin(ceil_div(*n_ptr, kSortTile), tiles_max);
    const int64_t words = ntile * nb;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int p = 0; p < passes; p++)
        for (int64_t i = i0; i < words; i += stride) status[p * tiles_max * nb + i] = 0ull;
    for (int64_t i = i0; i < (int64_t)passes * nb; i += stride) hist[i] = 0u;
    if (i0 == 0) *err = 0;
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_onesweep(const uint32_t* __restrict__ keys_in,
                                                           const int32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           int32_t* __restrict__ vals_out,
                                                           const int64_t* __restrict__ n_ptr, int shift,
                                                           const uint32_t* __restrict__ digit_base,
                                                           const uint32_t* __restrict__ uniform, int stay,
                                                           unsigned long long* __restrict__ status,
                                                           int32_t* __restrict__ err) {
    constexpr int NB = 1 << BITS;
    constexpr int PER = NB >= kSortThreads ? NB / kSortThreads : 1;   // digits per thread
    constexpr int ACT = NB / PER;                                     // threads owning digits
    __shared__ uint32_t s_hist[4][NB];      // per-wave digit counts, then each wave's offset inside the digit
    __shared__ uint32_t s_lstart[NB];       // first position of each digit in the tile
    __shared__ int32_t s_glob[NB];          // output index of a digit's first pair, less s_lstart
    __shared__ uint32_t s_part[kSortThreads / 64];
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ int32_t s_vals[kSortTile];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    for (int d = t; d < NB; d += kSortThreads) {
#pragma unroll
        for (int w = 0; w < 4; w++) s_hist[w][d] = 0;
    }
    __syncthreads();
    const int64_t n = *n_ptr;
    const int64_t b = blockIdx.x;
    if (b >= ceil_div(n, kSortTile)) return;
    if (*uniform) {     // every key has the same digit: the stable order is the input order
        if (stay) return;   // the caller reads the input buffers when this pass is uniform
        const int64_t e = imin(n, (b + 1) * kSortTile);
        for (int64_t i = b * kSortTile + t; i < e; i += kSortThreads) {
            keys_out[i] = keys_in[i];
            vals_out[i] = vals_in[i];
        }
        return;
    }
    uint32_t key[kSortItems];
    int32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t idx = b * kSortTile + (int64_t)wid * (kSortTile / 4) + r * 64 + lane;
        const bool active = idx < n;
        key[r] = active ? keys_in[idx] : 0u;
        val[r] = active ? vals_in[idx] : 0;
    }
    const int64_t start = b * kSortTile + (int64_t)wid * (kSortTile / 4);
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t idx = start + r * 64 + lane;
        const bool active = idx < n;
        const uint32_t d = (key[r] >> shift) & (NB - 1);
        const uint64_t peers = match_digit<BITS>(d, active);
        const uint64_t below = peers & ((1ull << lane) - 1ull);
        const uint32_t base = s_hist[wid][d];
        rank[r] = base + (uint32_t)__popcll(below);
        if (active && below == 0) s_hist[wid][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: offsets of the waves inside the digit, the tile's count, and its status word
    uint32_t tot[PER];
    uint32_t mine = 0;
    if (t < ACT) {
#pragma unroll
        for (int e = 0; e < PER; e++) {
            const int d = t * PER + e;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < 4; w++) {
                const uint32_t c = s_hist[w][d];
                s_hist[w][d] = run;
                run += c;
            }
            tot[e] = run;
            mine += run;
            st_publish(&status[b * NB + d], b == 0 ? kStPre : kStAgg, run);
        }
    }
    // exclusive scan of the tile's digit counts -> s_lstart
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_part[wid] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wid; w++) pre += s_part[w];
    if (t < ACT) {
        uint32_t x = pre + incl - mine;
#pragma unroll
        for (int e = 0; e < PER; e++) {
            s_lstart[t * PER + e] = x;
            x += tot[e];
        }
    }
    __syncthreads();
    // the tile's pairs in digit order in LDS (stable: waves, then rounds, then lanes)
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t idx = start + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & (NB - 1);
            const uint32_t pos = s_lstart[d] + s_hist[wid][d] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    // look-back: this digit's count over the tiles before b
    if (t < ACT) {
#pragma unroll
        for (int e = 0; e < PER; e++) {
            const int d = t * PER + e;
            uint32_t excl = 0;
            if (b > 0) {
                excl = lookback_excl(status + d, NB, b, err);
                st_publish(&status[b * NB + d], kStPre, excl + tot[e]);
            }
            s_glob[d] = (int32_t)(digit_base[d] + excl) - (int32_t)s_lstart[d];
        }
    }
    __syncthreads();
    const int64_t tile_n = imin(kSortTile, n - b * kSortTile);
    for (int64_t i = t; i < tile_n; i += kSortThreads) {
        const uint32_t k = s_keys[i];
        const int64_t o = (int64_t)s_glob[(k >> shift) & (NB - 1)] + i;
        keys_out[o] = k;
        vals_out[o] = s_vals[i];
    }
}

// Bit 1 of the caller's overflow word: some look-back gave up (results undefined).
__global__ void k_os_report(const int32_t* __restrict__ err, int32_t* __restrict__ overflow) {
    if (*err) *overflow |= 2;
}

// Workspace of the onesweep passes of one sort of at most `cap` pairs.
struct OsWs {
    unsigned long long* status;
    uint32_t* hist;
    uint32_t* uni;       // per pass: one digit holds every key
    int32_t* err;
    int64_t tiles_max;
};
size_t os_ws_bytes(int64_t cap, DigitPlan pl) {
    const int64_t tiles = imax(ceil_div(imax(cap, 1), kSortTile), 1);
    return align256((size_t)pl.passes * tiles * ((size_t)1 << pl.digit) * 8) +
           align256((size_t)kMaxSortPasses * ((size_t)1 << kOsMaxBits) * 4) + align256(kMaxSortPasses * 4) +
           align256(4);
}
OsWs os_carve(int64_t cap, DigitPlan pl, char* p) {
    OsWs w{};
    w.tiles_max = imax(ceil_div(imax(cap, 1), kSortTile), 1);
    size_t off = 0;
    w.status = (unsigned long long*)(p + off);
    off += align256((size_t)pl.passes * w.tiles_max * ((size_t)1 << pl.digit) * 8);
    w.hist = (uint32_t*)(p + off);
    off += align256((size_t)kMaxSortPasses * ((size_t)1 << kOsMaxBits) * 4);
    w.uni = (uint32_t*)(p + off);
    off += align256(kMaxSortPasses * 4);
    w.err = (int32_t*)(p + off);
    return w;
}

// Stable LSD sort of the *n_ptr (<= cap) pairs in (ka, va) by their low
// pl.passes * pl.digit key bits, ping-ponging with (kb, vb); the result
// lands in (ka, va) for an even number of passes, else in (kb, vb).
// uniform_high: keys whose high digits mostly agree (depth bits), counted with
// the wave-uniform shortcut.  last_may_stay: when the last pass's digit is one
// value for every key, that pass moves nothing and the result stays where the
// pass before left it; w.uni[passes - 1] tells the caller which.
hipError_t onesweep_sort(DigitPlan pl, uint32_t* ka, int32_t* va, uint32_t* kb, int32_t* vb, const int64_t* n_ptr,
                         int64_t cap, OsWs w, int32_t* overflow, bool uniform_high, bool last_may_stay,
                         hipStream_t s) {
    const int nb = 1 << pl.digit;
    k_os_clear<<<1024, 256, 0, s>>>(n_ptr, pl.passes, nb, w.tiles_max, w.status, w.hist, w.err);
    const unsigned hgrid = (unsigned)imax(1, imin(2048, ceil_div(imax(cap, 1), 256 * 16)));
    switch (pl.digit) {
#define PG_HIST(B)                                                                                     \
    case B:                                                                                            \
        if (uniform_high) k_os_hist<B, true><<<hgrid, 256, 0, s>>>(ka, n_ptr, pl.passes, w.hist);      \
        else k_os_hist<B, false><<<hgrid, 256, 0, s>>>(ka, n_ptr, pl.passes, w.hist);                  \
        break;
        PG_HIST(1) PG_HIST(2) PG_HIST(3) PG_HIST(4) PG_HIST(5) PG_HIST(6) PG_HIST(7) PG_HIST(8) PG_HIST(9)
#undef PG_HIST
        default: return hipErrorInvalidValue;
    }
    k_os_scan<<<1, 512, 0, s>>>(w.hist, pl.passes, nb, n_ptr, w.uni);
    const unsigned grid = (unsigned)w.tiles_max;
    for (int p = 0; p < pl.passes; p++) {
        unsigned long long* st = w.status + (int64_t)p * w.tiles_max * nb;
        const int stay = last_may_stay && p == pl.passes - 1 ? 1 : 0;
        switch (pl.digit) {
#define PG_PASS(B)                                                                                          \
    case B:                                                                                                 \
        k_onesweep<B><<<grid, kSortThreads, 0, s>>>(ka, va, kb, vb, n_ptr, p * pl.digit, w.hist + p * nb,    \
                                                   w.uni + p, stay, st, w.err);                             \
        break;
            PG_PASS(1) PG_PASS(2) PG_PASS(3) PG_PASS(4) PG_PASS(5) PG_PASS(6) PG_PASS(7) PG_PASS(8) PG_PASS(9)
#undef PG_PASS
            default: return hipErrorInvalidValue;
        }
        uint32_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (overflow) k_os_report<<<1, 1, 0, s>>>(w.err, overflow);
    return hipGetLastError();
}

// [start, end) of every tile from the sorted keys: a tile starts where the key
// differs from its predecessor, which is also where the previous tile ends.
// Four consecutive keys per thread, over a fixed grid that strides through
// the device-side count (a grid sized for the capacity was mostly empty
// groups); the predecessor of a thread's first key is the neighbouring lane's
// last (only the first lane of a wave loads it), so every key is read once.
constexpr int kRangeGrid = 4096;
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const int64_t* __restrict__ misc,
                                                int32_t* __restrict__ ranges) {
    const int64_t I = misc[1];
    const int64_t nq = (I + 3) / 4;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < nq; base += (int64_t)gridDim.x * 256) {
        const int64_t i0 = 4 * (base + threadIdx.x);
        uint32_t k[4];
#pragma unroll
        for (int j = 0; j < 4; j++) k[j] = i0 + j < I ? keys[i0 + j] : 0u;
        uint32_t prev = __shfl_up(k[3], 1, 64);
        if ((threadIdx.x & 63) == 0 && i0 > 0 && i0 < I) prev = keys[i0 - 1];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t i = i0 + j;
            if (i >= I) break;
            const uint32_t p = j == 0 ? prev : k[j - 1];
            if (i == 0) {
                ranges[2 * (int64_t)k[j]] = 0;
            } else if (p != k[j]) {
                ranges[2 * (int64_t)k[j]] = (int32_t)i;
                ranges[2 * (int64_t)p + 1] = (int32_t)i;
            }
            if (i == I - 1) ranges[2 * (int64_t)k[j] + 1] = (int32_t)I;
        }
    }
}

// ---------------------------------------------------------------- tile dispatch order
// The compositing kernels run one work-group per tile, and tiles differ in
// cost by their list lengths.  Dispatching the longest lists first (a
// longest-processing-time-first schedule) shortens the tail of those
// launches, where a few long tiles would otherwise run on an emptying chip.
// The order is coarse: 64 classes of list length, four per octave, longest
// class first.  Inside a class, tiles keep their index order and are dealt to
// the XCDs in contiguous runs: the dispatcher hands work-group b to XCD b mod
// 8, so the slots of a class that land on XCD x receive one run of
// neighbouring tiles, which share Gaussians and so their records in that
// XCD's L2.  The order is deterministic and results do not depend on it.
__device__ __forceinline__ int order_class(int32_t len) {
    const uint32_t b = __float_as_uint((float)(len > 0 ? len : 0) + 1.0f);
    const int c = 4 * ((int)((b >> 23) & 0xffu) - 127) + (int)((b >> 21) & 3u);   // 4 log2(len + 1), floored
    return kOrderClasses - 1 - (c < 0 ? 0 : (c < kOrderClasses - 1 ? c : kOrderClasses - 1));
}

// Per work-group of kOrderBlk consecutive tiles: the tile count of each class.
__global__ __launch_bounds__(kOrderBlk) void k_order_count(const int2* __restrict__ ranges, int64_t n_tiles,
                                                           int32_t* __restrict__ cnt) {
    __shared__ int32_t s_cnt[kOrderClasses];
    if (threadIdx.x < kOrderClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kOrderBlk + threadIdx.x;
    if (t < n_tiles) {
        const int2 r = ranges[t];
        atomicAdd(&s_cnt[order_class(r.y - r.x)], 1);     // counts only: order-free
    }
    __syncthreads();
    if (threadIdx.x < kOrderClasses) cnt[(int64_t)blockIdx.x * kOrderClasses + threadIdx.x] = s_cnt[threadIdx.x];
}

// Class-major exclusive scan of the counts (one work-group of 1024 threads):
// base[w][c] = tiles of the classes before c + tiles of class c in groups
// before w; cls[c] = first slot of class c, cls[kOrderClasses + c] = its size.
constexpr int kOrderSeg = 1024 / kOrderClasses;     // threads per class in the scan
__global__ __launch_bounds__(1024) void k_order_scan(const int32_t* __restrict__ cnt, int64_t n_groups,
                                                     int32_t* __restrict__ base, int32_t* __restrict__ cls) {
    __shared__ int32_t s_part[kOrderClasses][kOrderSeg];
    __shared__ int32_t s_first[kOrderClasses];
    // thread (c, k): class c of the k-th run of groups; a wave reads whole rows
    // of 64 class counts, and the loads of a run are independent
    const int c = threadIdx.x % kOrderClasses, k = threadIdx.x / kOrderClasses;
    const int64_t per = ceil_div(n_groups, kOrderSeg);
    const int64_t w0 = imin(n_groups, k * per), w1 = imin(n_groups, w0 + per);
    int32_t sum = 0;
#pragma unroll 8
    for (int64_t w = w0; w < w1; w++) sum += cnt[w * kOrderClasses + c];
    s_part[c][k] = sum;
    __syncthreads();
    if (threadIdx.x < 64) {     // one wave: class totals and their exclusive scan
        int32_t tot = 0;
        for (int j = 0; j < kOrderSeg; j++) tot += s_part[threadIdx.x][j];
        int32_t incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(incl, o, 64);
            if ((int)threadIdx.x >= o) incl += u;
        }
        s_first[threadIdx.x] = incl - tot;
        cls[threadIdx.x] = incl - tot;
        cls[kOrderClasses + threadIdx.x] = tot;
    }
    __syncthreads();
    int32_t run = s_first[c];
    for (int j = 0; j < k; j++) run += s_part[c][j];
#pragma unroll 8
    for (int64_t w = w0; w < w1; w++) {
        base[w * kOrderClasses + c] = run;
        run += cnt[w * kOrderClasses + c];
    }
}

// Dispatch slot of the rank-r tile (in index order) of a class holding slots
// [o, o + n): XCD x receives the ranks [R_x, R_x + m_x), where m_x counts the
// class's slots s with s mod 8 = x and R_x those of the XCDs before x.
__device__ __forceinline__ int64_t order_slot(int64_t o, int64_t n, int64_t r) {
    int64_t R = 0;
    for (int x = 0; x < 8; x++) {
        const int64_t f = o + ((x - (o & 7)) & 7);        // first slot of the class on XCD x
        const int64_t m = f < o + n ? (o + n - f + 7) / 8 : 0;
        if (r < R + m) return f + 8 * (r - R);
        R += m;
    }
    return -1;     // r >= n: not reached for ranks of the class
}

__global__ __launch_bounds__(kOrderBlk) void k_order_place(const int2* __restrict__ ranges, int64_t n_tiles,
                                                           const int32_t* __restrict__ base,
                                                           const int32_t* __restrict__ cls,
                                                           int32_t* __restrict__ order) {
    __shared__ uint32_t s_hist[kOrderBlk / 64][kOrderClasses];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = lane; c < kOrderClasses; c += 64) s_hist[wid][c] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kOrderBlk + threadIdx.x;
    const bool active = t < n_tiles;
    int c = 0;
    if (active) {
        const int2 r = ranges[t];
        c = order_class(r.y - r.x);
    }
    // rank among the lanes of this wave with the same class, then among earlier waves
    const uint64_t peers = match_digit<6>((uint32_t)c, active);
    const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    if (active && below == 0) s_hist[wid][c] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (!active) return;
    uint32_t rank = below;
    for (int w = 0; w < wid; w++) rank += s_hist[w][c];
    const int64_t o = cls[c], n = cls[kOrderClasses + c];
    const int64_t r = (int64_t)base[(int64_t)blockIdx.x * kOrderClasses + c] - o + rank;
    const int64_t slot = order_slot(o, n, r);
    if (slot >= 0 && slot < n_tiles) order[slot] = (int32_t)t;
}

hipError_t launch_tile_order(const int32_t* ranges, int64_t n_tiles, int32_t* cnt, int32_t* base, int32_t* cls,
                             int32_t* order, hipStream_t s) {
    if (!order || n_tiles == 0) return hipSuccess;
    const int64_t groups = ceil_div(n_tiles, kOrderBlk);
    const int2* rg = reinterpret_cast<const int2*>(ranges);
    k_order_count<<<(unsigned)groups, kOrderBlk, 0, s>>>(rg, n_tiles, cnt);
    k_order_scan<<<1, 1024, 0, s>>>(cnt, groups, base, cls);
    k_order_place<<<(unsigned)groups, kOrderBlk, 0, s>>>(rg, n_tiles, base, cls, order);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- generic stable pair sort
// The same LSD passes for other parts of the library: n (read on the device,
// at most cap) uint32 keys whose low `bits` bits matter, with int32 values,
// ping-ponged between the two buffer pairs; *out_keys / *out_vals name the
// pair that holds the result.
namespace {
}  // namespace

size_t sort_pairs_ws_bytes(int64_t cap, int bits) {
    return os_ws_bytes(cap, digit_plan(bits, kDepthDigitBits));
}

hipError_t sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, const int64_t* n_dev,
                      int64_t cap, int bits, void* ws, uint32_t** out_keys, int32_t** out_vals, hipStream_t s) {
    const DigitPlan pl = digit_plan(bits, kDepthDigitBits);
    const hipError_t e = onesweep_sort(pl, keys, vals, keys_alt, vals_alt, n_dev, cap, os_carve(cap, pl, (char*)ws),
                                       nullptr, true, false, s);
    const bool even = pl.passes % 2 == 0;
    *out_keys = even ? keys : keys_alt;
    *out_vals = even ? vals : vals_alt;
    return e;
}

size_t sort_ws_bytes(const pg_views* v, int64_t cap) {
    size_t total = 0;
    carve(v, cap, nullptr, &total);
    return total;
}

hipError_t launch_bin_sort(const pg_views* v, const pg_bin* bins, const pg_tile_set* tiles, int64_t cap,
                           uint32_t* keys, int32_t* values,
                           int32_t* ranges, int32_t* tile_order, int32_t* inst_first, int64_t* n_inst_dev,
                           int32_t* overflow_dev, void* ws, hipStream_t s) {
    const SortPlan pl = plan_for(v);
    SortWs w = carve(v, cap, ws, nullptr);
    const int64_t nb = n_blocks(v);
    hipError_t e = fill_u32(ranges, 0u, 2 * v->n_tiles, s);
    if (e != hipSuccess) return e;
    e = fill_u32(overflow_dev, 0u, 1, s);      // bit 0: capacity overflow; bit 1: a radix pass gave up waiting
    if (e != hipSuccess) return e;
    if (v->n_gv == 0) {
        e = fill_u32(w.misc, 0u, 16, s);
        if (e != hipSuccess) return e;
        e = fill_u32(n_inst_dev, 0u, 2, s);
        if (e != hipSuccess) return e;
        k_post_count<<<1, 1, 0, s>>>(n_inst_dev, cap, overflow_dev, w.misc);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_tile_order(ranges, v->n_tiles, w.order_cnt, w.order_base, w.order_cls, tile_order, s);
    }
    // 1. compact surviving records in (view, id) order, keyed by depth; slot offsets in the same order
    k_valid_count<<<(unsigned)nb, kBlk, 0, s>>>(bins, v->n_gv, w.blk_a, w.blk_b);
    e = scan_i64(w.blk_a, w.blk_a_off, nullptr, 0, nb, w.misc + 0, w.scan_tmp, s);
    if (e != hipSuccess) return e;
    e = scan_i64(w.blk_b, w.blk_b_off, nullptr, 0, nb, w.misc + 4, w.scan_tmp, s);
    if (e != hipSuccess) return e;
    k_compact<<<(unsigned)nb, kBlk, 0, s>>>(bins, v->n_gv, w.blk_a_off, w.blk_b_off, w.rk0, w.rv0, inst_first);
    // 2. stable LSD sort of the records by depth
    // (when the last digit is one value for every key, that pass moves nothing: the
    // records stay in the buffer the pass before wrote, and its flag says so)
    const OsWs dws = os_carve(v->n_gv, pl.depth, w.os);
    e = onesweep_sort(pl.depth, w.rk0, w.rv0, w.rk1, w.rv1, w.misc + 0, v->n_gv, dws, overflow_dev, true, true, s);
    if (e != hipSuccess) return e;
    const int32_t* rva = pl.depth.passes % 2 == 0 ? w.rv0 : w.rv1;
    const int32_t* rvb = pl.depth.passes % 2 == 0 ? w.rv1 : w.rv0;
    const uint32_t* stayed = dws.uni + pl.depth.passes - 1;
    // 3. instance offsets in sorted-record order; overflow check
    k_sorted_count<<<(unsigned)nb, kBlk, 0, s>>>(tiles, rva, rvb, stayed, w.misc, w.blk_a, w.stiles);
    e = scan_i64(w.blk_a, w.blk_a_off, nullptr, 0, nb, n_inst_dev, w.scan_tmp, s);
    if (e != hipSuccess) return e;
    k_post_count<<<1, 1, 0, s>>>(n_inst_dev, cap, overflow_dev, w.misc);
    // 4. emit (tile, gv) in record order into the buffer that makes the last tile pass land in the caller's arrays
    const bool even = pl.tile.passes % 2 == 0;
    uint32_t* ta = even ? keys : w.tk_alt;
    int32_t* tva = even ? values : w.tv_alt;
    uint32_t* tb = even ? w.tk_alt : keys;
    int32_t* tvb = even ? w.tv_alt : values;
    k_emit<<<(unsigned)nb, kBlk, 0, s>>>(w.stiles, rva, rvb, stayed, v->n_gauss, v->d_views, w.blk_a_off, w.misc, ta,
                                         tva);
    // 5. stable LSD sort of the instances by tile id (its workspace overlaps the depth sort's, whose flag
    // the emission has read by then)
    e = onesweep_sort(pl.tile, ta, tva, tb, tvb, w.misc + 1, cap, os_carve(cap, pl.tile, w.os), overflow_dev, false,
                      false, s);
    if (e != hipSuccess) return e;
    k_ranges<<<(unsigned)imax(1, imin(kRangeGrid, ceil_div(cap, 256))), 256, 0, s>>>(keys, w.misc, ranges);
    return launch_tile_order(ranges, v->n_tiles, w.order_cnt, w.order_base, w.order_cls, tile_order, s);
}

}  // namespace pg
