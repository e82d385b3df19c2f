// a1 -- atlas fetch: stream-compaction of occupied texels and a gather of
// their raw channels into per-Gaussian planes.
//
// Occupied texels in row-major order are the Gaussians of every frame of the
// window (one atlas per frame, shared occupancy); the rank of a texel is the
// Gaussian id ("Fitting UV Maps Directly", Sec. 4.2; atlas layout, Sec. 4.1).
// HBM-bound: one byte per texel for occupancy plus 4 C bytes per Gaussian and
// frame read and written once; reads along a row of the atlas are coalesced.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kThreads = 256;
constexpr int kBytes = 16;                    // occupancy bytes per thread
constexpr int kTile = kThreads * kBytes;      // texels per work-group

__device__ __forceinline__ int nonzero_bytes(uint32_t w) {
    uint32_t t = w | (w >> 4);
    t |= t >> 2;
    t |= t >> 1;
    return __popc(t & 0x01010101u);
}

__device__ __forceinline__ void load16(const uint8_t* occ, int64_t beg, int64_t n, uint8_t b[kBytes]) {
    if (beg + kBytes <= n && ((reinterpret_cast<uintptr_t>(occ + beg) & 15) == 0)) {
        uint4 v = *reinterpret_cast<const uint4*>(occ + beg);
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < kBytes; k++) b[k] = (uint8_t)((w[k >> 2] >> (8 * (k & 3))) & 0xff);
    } else {
#pragma unroll
        for (int k = 0; k < kBytes; k++) b[k] = (beg + k < n) ? occ[beg + k] : 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_occ_count(const uint8_t* occ, int64_t n, int32_t* block_counts) {
    __shared__ int s[kThreads / 64];
    const int64_t beg = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kBytes;
    int c = 0;
    if (beg + kBytes <= n && ((reinterpret_cast<uintptr_t>(occ + beg) & 15) == 0)) {
        uint4 v = *reinterpret_cast<const uint4*>(occ + beg);
        c = nonzero_bytes(v.x) + nonzero_bytes(v.y) + nonzero_bytes(v.z) + nonzero_bytes(v.w);
    } else {
        for (int k = 0; k < kBytes; k++) c += (beg + k < n && occ[beg + k]) ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kThreads / 64; w++) tot += s[w];
        block_counts[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(kThreads) void k_occ_ids(const uint8_t* occ, int64_t n, const int64_t* block_off,
                                                      int64_t n_cap, int32_t* gauss_texel,
                                                      int32_t* texel_gauss) {
    __shared__ int s_warp[kThreads / 64];
    const int64_t beg = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kBytes;
    uint8_t b[kBytes];
    load16(occ, beg, n, b);
    int c = 0;
#pragma unroll
    for (int k = 0; k < kBytes; k++) c += b[k] ? 1 : 0;
    // exclusive prefix of c over the work-group
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int v = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) s_warp[wid] = v;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; w++) before += s_warp[w];
    int64_t id = block_off[blockIdx.x] + before + v - c;
#pragma unroll
    for (int k = 0; k < kBytes; k++) {
        const int64_t slot = beg + k;
        if (slot >= n) break;
        if (b[k]) {
            if (id < n_cap) gauss_texel[id] = (int32_t)slot;
            texel_gauss[slot] = (id < n_cap) ? (int32_t)id : -1;
            id++;
        } else {
            texel_gauss[slot] = -1;
        }
    }
}

__global__ __launch_bounds__(256) void k_gather(const float* atlas, int32_t F, int32_t C, int64_t HW,
                                                const int32_t* gauss_texel, const int64_t* n_dev, int64_t n_cap,
                                                float* params) {
    const int64_t n = imin(*n_dev, n_cap);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t texel = gauss_texel[i];
    for (int32_t fc = 0; fc < F * C; fc++) params[(int64_t)fc * n_cap + i] = atlas[(int64_t)fc * HW + texel];
}

}  // namespace

size_t fetch_ws_bytes(int32_t H, int32_t W) {
    const int64_t nb = ceil_div((int64_t)H * W, kTile);
    return align256(nb * 4) + align256(nb * 8) + align256(kScanTmpWords * 8);
}

hipError_t launch_fetch(const float* atlas, const uint8_t* occ, int32_t F, int32_t C, int32_t H, int32_t W,
                        int64_t n_cap, int32_t* gauss_texel, int32_t* texel_gauss, float* params,
                        int64_t* n_gauss_dev, void* ws, hipStream_t s) {
    const int64_t HW = (int64_t)H * W;
    const int64_t nb = ceil_div(HW, kTile);
    char* p = (char*)ws;
    int32_t* counts = (int32_t*)p;
    p += align256(nb * 4);
    int64_t* offs = (int64_t*)p;
    p += align256(nb * 8);
    int64_t* tmp = (int64_t*)p;
    k_occ_count<<<(unsigned)nb, kThreads, 0, s>>>(occ, HW, counts);
    hipError_t e = scan_i32_as_i64(counts, offs, nullptr, 0, nb, n_gauss_dev, tmp, s);
    if (e != hipSuccess) return e;
    k_occ_ids<<<(unsigned)nb, kThreads, 0, s>>>(occ, HW, offs, n_cap, gauss_texel, texel_gauss);
    if (n_cap > 0)
        k_gather<<<(unsigned)ceil_div(n_cap, 256), 256, 0, s>>>(atlas, F, C, HW, gauss_texel, n_gauss_dev, n_cap,
                                                               params);
    return hipGetLastError();
}

}  // namespace pg
