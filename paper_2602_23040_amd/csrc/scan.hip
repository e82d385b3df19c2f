// Device-length exclusive scans and fill kernels.
//
// Every length may live in device memory (written by an earlier kernel of
// the same stream), so that whole call chains run without host round trips
// and can be captured in a HIP graph.  The scans use a fixed grid of
// kScanBlocks work-groups: reduce per contiguous chunk, scan the chunk sums
// in one work-group, then rescan each chunk with its offset.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

__global__ void k_fill_u32_dev(uint32_t* p, uint32_t value, const int64_t* n_dev, int64_t n_max, int64_t mul) {
    const int64_t n = imin(*n_dev, n_max) * mul;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

__device__ __forceinline__ int64_t scan_length(const int64_t* n_dev, int64_t n_mul, int64_t n_host) {
    return n_dev ? (*n_dev) * n_mul : n_host;
}

// Inclusive scan across a 256-thread work-group; returns this thread's
// inclusive prefix and the group total.
__device__ __forceinline__ int64_t block_inclusive(int64_t v, int64_t* s_warp, int64_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_warp[wid] = v;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; w++) {
        int64_t x = s_warp[w];
        before += (w < wid) ? x : 0;
        all += x;
    }
    __syncthreads();
    *total = all;
    return v + before;
}

template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_chunk_reduce(const Tin* in, const int64_t* n_dev, int64_t n_mul,
                                                           int64_t n_host, int64_t* block_tmp) {
    __shared__ int64_t s_warp[kThreads / 64];
    const int64_t n = scan_length(n_dev, n_mul, n_host);
    const int64_t chunk = ceil_div(n, kScanBlocks);
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = imin(n, beg + chunk);
    int64_t acc = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) acc += (int64_t)in[i];
    int64_t tot;
    block_inclusive(acc, s_warp, &tot);
    if (threadIdx.x == 0) block_tmp[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlocks) void k_scan_chunks(int64_t* block_tmp, int64_t* total_out) {
    __shared__ int64_t s[kScanBlocks];
    const int t = threadIdx.x;
    s[t] = block_tmp[t];
    __syncthreads();
    for (int o = 1; o < kScanBlocks; o <<= 1) {
        int64_t u = (t >= o) ? s[t - o] : 0;
        __syncthreads();
        s[t] += u;
        __syncthreads();
    }
    block_tmp[t] = (t == 0) ? 0 : s[t - 1];
    if (t == kScanBlocks - 1) {
        block_tmp[kScanBlocks] = s[t];
        if (total_out) *total_out = s[t];
    }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void k_chunk_scan(const Tin* in, Tout* out, const int64_t* n_dev,
                                                         int64_t n_mul, int64_t n_host, const int64_t* block_tmp) {
    __shared__ int64_t s_warp[kThreads / 64];
    const int64_t n = scan_length(n_dev, n_mul, n_host);
    const int64_t chunk = ceil_div(n, kScanBlocks);
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = imin(n, beg + chunk);
    int64_t run = block_tmp[blockIdx.x];
    for (int64_t base = beg; base < end; base += (int64_t)kThreads * kItems) {
        int64_t v[kItems];
        int64_t sum = 0;
        const int64_t my = base + (int64_t)threadIdx.x * kItems;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            v[k] = (my + k < end) ? (int64_t)in[my + k] : 0;
            sum += v[k];
        }
        int64_t tot;
        int64_t incl = block_inclusive(sum, s_warp, &tot);
        int64_t x = run + incl - sum;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            if (my + k < end) out[my + k] = (Tout)x;
            x += v[k];
        }
        run += tot;
    }
}

template <typename Tin, typename Tout>
hipError_t scan_impl(const Tin* in, Tout* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                     int64_t* total_out, int64_t* block_tmp, hipStream_t s) {
    k_chunk_reduce<Tin><<<kScanBlocks, kThreads, 0, s>>>(in, n_dev, n_mul, n_host, block_tmp);
    k_scan_chunks<<<1, kScanBlocks, 0, s>>>(block_tmp, total_out);
    k_chunk_scan<Tin, Tout><<<kScanBlocks, kThreads, 0, s>>>(in, out, n_dev, n_mul, n_host, block_tmp);
    return hipGetLastError();
}

}  // namespace

hipError_t fill_u32(void* p, uint32_t value, int64_t n_words, hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    int64_t blocks = imin(ceil_div(n_words, 256), 4096);
    k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>((uint32_t*)p, value, n_words);
    return hipGetLastError();
}

// Fill of min(*n_dev, n_max) * mul words, the count read on the device.
hipError_t fill_u32_dev(void* p, uint32_t value, const int64_t* n_dev, int64_t n_max, int64_t mul, hipStream_t s) {
    k_fill_u32_dev<<<4096, 256, 0, s>>>((uint32_t*)p, value, n_dev, n_max, mul);
    return hipGetLastError();
}

hipError_t scan_i64(const int64_t* in, int64_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                    int64_t* total_out, int64_t* block_tmp, hipStream_t s) {
    return scan_impl<int64_t, int64_t>(in, out, n_dev, n_mul, n_host, total_out, block_tmp, s);
}

hipError_t scan_i32_as_i64(const int32_t* in, int64_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                           int64_t* total_out, int64_t* block_tmp, hipStream_t s) {
    return scan_impl<int32_t, int64_t>(in, out, n_dev, n_mul, n_host, total_out, block_tmp, s);
}

// int32 -> int32 variant for radix digit counts (totals stay below 2^31).
hipError_t scan_i32(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n_mul, int64_t n_host,
                    int64_t* total_out, int64_t* block_tmp, hipStream_t s) {
    return scan_impl<int32_t, int32_t>(in, out, n_dev, n_mul, n_host, total_out, block_tmp, s);
}

}  // namespace pg
