// Low-precision optimisation (LPO): the uniform K-bit fake quantiser the
// renderer consumes in place of the FP32 master texel values (Sec. 4.3 LPO
// paragraph; supplementary low-precision training section), with the
// per-channel min/max scale of the supplementary video-coding section.
//
// Per channel c with K = bits[c] > 0, over the fetched values of every frame:
//   lo, hi = min, max;  delta = (hi - lo) / (2^K - 1);
//   code = clamp(rint((v - lo) / delta), 0, 2^K - 1);  proxy = lo + code delta.
// The code is an integer that floating point decides, so every step is one
// correctly rounded FP32 operation (no contraction; rint ties to even), which
// an independent implementation in the same order reproduces bit for bit.
// The straight-through estimator makes the adjoint of the quantiser the
// identity: the texel gradient at the proxy is the master values' gradient.
//
// Kernels (HBM-bound, 12 bytes per quantised value: two reads, one write):
//   k_quant_minmax  a fixed grid of work-groups per channel, each reducing a
//                   strided share of the channel to a (min, max) partial
//   k_quant_range   the partials of a channel -> (lo, hi)
//   k_quant_apply   proxy (in place) and optional 16-bit code per value
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kQThreads = 256;

struct QuantBits {
    int32_t b[kMaxQuantChannels];
};

__device__ __forceinline__ void wave_minmax(float& lo, float& hi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
}

__global__ __launch_bounds__(kQThreads) void k_quant_minmax(const float* __restrict__ params,
                                                            const int64_t* __restrict__ n_dev, int64_t n_cap,
                                                            int32_t F, int32_t C, QuantBits bits,
                                                            float* __restrict__ partial) {
    __shared__ float s_lo[kQThreads / 64], s_hi[kQThreads / 64];
    const int c = blockIdx.y;
    if (bits.b[c] <= 0) return;   // uniform over the work-group
    const int64_t n = imin(*n_dev, n_cap);
    float lo = INFINITY, hi = -INFINITY;
    for (int32_t f = 0; f < F; f++) {
        const float* row = params + ((int64_t)f * C + c) * n_cap;
        for (int64_t i = (int64_t)blockIdx.x * kQThreads + threadIdx.x; i < n; i += (int64_t)kQuantBlocks * kQThreads) {
            const float v = row[i];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    wave_minmax(lo, hi);
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kQThreads / 64; w++) {
            lo = fminf(lo, s_lo[w]);
            hi = fmaxf(hi, s_hi[w]);
        }
        partial[((int64_t)c * kQuantBlocks + blockIdx.x) * 2] = lo;
        partial[((int64_t)c * kQuantBlocks + blockIdx.x) * 2 + 1] = hi;
    }
}

// range[c] = (lo, hi); (0, 0) for channels left alone or with no value.
__global__ __launch_bounds__(kQuantBlocks) void k_quant_range(const float* __restrict__ partial, QuantBits bits,
                                                              float* __restrict__ range) {
    __shared__ float s_lo[kQuantBlocks / 64], s_hi[kQuantBlocks / 64];
    const int c = blockIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    if (bits.b[c] > 0) {
        lo = partial[((int64_t)c * kQuantBlocks + threadIdx.x) * 2];
        hi = partial[((int64_t)c * kQuantBlocks + threadIdx.x) * 2 + 1];
    }
    wave_minmax(lo, hi);
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kQuantBlocks / 64; w++) {
            lo = fminf(lo, s_lo[w]);
            hi = fmaxf(hi, s_hi[w]);
        }
        const bool any = lo <= hi;
        range[2 * c] = any ? lo : 0.0f;
        range[2 * c + 1] = any ? hi : 0.0f;
    }
}

__global__ __launch_bounds__(kQThreads) void k_quant_apply(float* __restrict__ params, const int64_t* __restrict__ n_dev,
                                                           int64_t n_cap, int32_t C, QuantBits bits,
                                                           const float* __restrict__ range,
                                                           uint16_t* __restrict__ codes) {
    const int32_t fc = blockIdx.y;
    const int c = fc % C;
    const int64_t n = imin(*n_dev, n_cap);
    const int64_t i = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t e = (int64_t)fc * n_cap + i;
    const int K = bits.b[c];
    if (K <= 0) {
        if (codes) codes[e] = 0;
        return;
    }
    const float lo = range[2 * c], hi = range[2 * c + 1];
    const float levels = (float)((1 << K) - 1);
    const float delta = (hi - lo) / levels;
    float k = 0.0f;
    if (delta > 0.0f) {
        const float d = params[e] - lo;
        k = rintf(d / delta);
        k = fminf(fmaxf(k, 0.0f), levels);
    }
    const float step = k * delta;
    params[e] = lo + step;
    if (codes) codes[e] = (uint16_t)k;
}

}  // namespace

hipError_t launch_fake_quant(float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C,
                             const int32_t* bits, float* range, uint16_t* codes, float* partial, hipStream_t s) {
    QuantBits qb{};
    for (int c = 0; c < C; c++) qb.b[c] = bits[c];
    k_quant_minmax<<<dim3(kQuantBlocks, (unsigned)C), kQThreads, 0, s>>>(params, n_dev, n_cap, F, C, qb, partial);
    k_quant_range<<<(unsigned)C, kQuantBlocks, 0, s>>>(partial, qb, range);
    if (n_cap > 0)
        k_quant_apply<<<dim3((unsigned)ceil_div(n_cap, kQThreads), (unsigned)(F * C)), kQThreads, 0, s>>>(
            params, n_dev, n_cap, C, qb, range, codes);
    return hipGetLastError();
}

}  // namespace pg
