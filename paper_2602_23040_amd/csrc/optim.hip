// a4' (L1 photometric term) and a6 (sparse Adam on the atlas).
//
// L1: L = mean |image - target| and dL/dimage = sign(image - target) / n
// (Sec. 4.2 "Objective", lambda_ssim = 0).  The sum is reduced in a fixed
// order (fixed grid, per-group partials in FP64, one final group), so the
// loss value is deterministic.  HBM-bound: 12 bytes per element.
//
// Adam: textbook update with bias correction on the FP32 master atlas,
// restricted to texels whose Gaussian was drawn in at least one view this
// step ("Sparse Adam", Sec. 4.3 LPO paragraph).  HBM-bound: 28 bytes per
// updated element (atlas, m, v read and written, gradient read).
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kLossBlocks = 1024;

// VEC: the three arrays are 16-byte aligned and each thread moves four
// elements per load and store (the streaming rate of 4-byte accesses was
// ~4.3 TB/s); the last n mod 4 elements take the scalar loop.
template <bool VEC>
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt, int64_t n,
                                            float* __restrict__ g, double* __restrict__ partial) {
    __shared__ double s[4];
    const float inv = (float)(1.0 / (double)n);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t done = 0;
    if (VEC) {
        const int64_t n4 = n / 4;
        const float4* a4 = reinterpret_cast<const float4*>(img);
        const float4* b4 = reinterpret_cast<const float4*>(tgt);
        float4* g4 = reinterpret_cast<float4*>(g);
        for (int64_t q = t0; q < n4; q += stride) {
            const float4 a = a4[q], b = b4[q];
            const float d[4] = {a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w};
            float o[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                acc += (double)fabsf(d[j]);
                o[j] = d[j] > 0.0f ? inv : (d[j] < 0.0f ? -inv : 0.0f);
            }
            g4[q] = make_float4(o[0], o[1], o[2], o[3]);
        }
        done = 4 * n4;
    }
    for (int64_t i = done + t0; i < n; i += stride) {
        const float d = img[i] - tgt[i];
        acc += (double)fabsf(d);
        g[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ __launch_bounds__(kLossBlocks) void k_l1_final(const double* __restrict__ partial, int64_t n,
                                                          float* __restrict__ loss) {
    __shared__ double s[kLossBlocks];
    s[threadIdx.x] = partial[threadIdx.x];
    __syncthreads();
    for (int o = kLossBlocks / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] / (double)n);
}

// The loss value from the compositing adjoint's per-tile sums of |image -
// target| (the L1 term formed inside the adjoint): thread t adds tiles t,
// t + 1024, ... in order, then a fixed tree, so the value is deterministic.
__global__ __launch_bounds__(kLossBlocks) void k_l1_tiles(const double* __restrict__ tile_loss, int64_t n_tiles,
                                                          int64_t n, float* __restrict__ loss) {
    __shared__ double s[kLossBlocks];
    double a = 0.0;
    // unrolled so that eight loads are in flight; the additions keep their order
#pragma unroll 8
    for (int64_t t = threadIdx.x; t < n_tiles; t += kLossBlocks) a += tile_loss[t];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = kLossBlocks / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] / (double)n);
}

// One Adam update of element (p, g, m, v); the same expression for every
// element and both launch shapes below.
__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                          float eps, float inv_c1, float inv_c2) {
    const float mm = b1 * m + (1.0f - b1) * g;
    const float vv = b2 * v + (1.0f - b2) * g * g;
    m = mm;
    v = vv;
    p = p - lr * (mm * inv_c1) / (sqrtf(vv * inv_c2) + eps);
}

__device__ __forceinline__ void bias_corrections(const int32_t* step_dev, float b1, float b2, float& inv_c1,
                                                 float& inv_c2) {
    if (step_dev) {   // bias correction of the device-counted step
        const double t = (double)*step_dev;
        inv_c1 = (float)(1.0 / (1.0 - pow((double)b1, t)));
        inv_c2 = (float)(1.0 / (1.0 - pow((double)b2, t)));
    }
}

// Texel-major sparse Adam: a thread owns TPT consecutive texels of one frame
// (blockIdx.y), looks their Gaussians and visibility up once, and walks the
// C channel planes; texels whose Gaussian is not visible read and write
// nothing.  VEC (TPT = 4): the four texels' channel values move as one
// 16-byte access (planes 16-byte aligned: H W % 4 == 0 and aligned buffers);
// then only planes where all four are invisible are skipped, and invisible
// lanes of a visible quad are written back unchanged.
template <bool VEC>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const uint8_t* __restrict__ visible,
                                              const int32_t* __restrict__ texel_gauss, int64_t N, int32_t C,
                                              int64_t HW, float lr, float b1, float b2, float eps, float inv_c1,
                                              float inv_c2, const int32_t* __restrict__ step_dev) {
    constexpr int TPT = VEC ? 4 : 1;
    bias_corrections(step_dev, b1, b2, inv_c1, inv_c2);
    const int64_t f = blockIdx.y;
    const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * TPT;
    if (t0 >= HW) return;
    bool on[TPT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < TPT; k++) {
        const int32_t id = (t0 + k < HW) ? texel_gauss[t0 + k] : -1;
        on[k] = id >= 0 && visible[f * N + id] != 0;
        any |= on[k];
    }
    if (!any) return;
    const int64_t plane0 = f * (int64_t)C * HW + t0;
    if (VEC) {
        // channels in groups of CG: every load of a group is issued before its
        // arithmetic, so each wave keeps 4 CG 16-byte loads in flight
        constexpr int CG = 4;
        auto group = [&](const int32_t c0, const int ng) __attribute__((always_inline)) {
            float4 gr[CG], pp[CG], mm[CG], vv[CG];
#pragma unroll
            for (int k = 0; k < CG; k++) {
                if (k >= ng) break;
                const int64_t e = plane0 + (int64_t)(c0 + k) * HW;
                gr[k] = *reinterpret_cast<const float4*>(g + e);
                pp[k] = *reinterpret_cast<const float4*>(p + e);
                mm[k] = *reinterpret_cast<const float4*>(m + e);
                vv[k] = *reinterpret_cast<const float4*>(v + e);
            }
#pragma unroll
            for (int k = 0; k < CG; k++) {
                if (k >= ng) break;
                if (on[0]) adam_elem(pp[k].x, gr[k].x, mm[k].x, vv[k].x, lr, b1, b2, eps, inv_c1, inv_c2);
                if (on[1]) adam_elem(pp[k].y, gr[k].y, mm[k].y, vv[k].y, lr, b1, b2, eps, inv_c1, inv_c2);
                if (on[2]) adam_elem(pp[k].z, gr[k].z, mm[k].z, vv[k].z, lr, b1, b2, eps, inv_c1, inv_c2);
                if (on[3]) adam_elem(pp[k].w, gr[k].w, mm[k].w, vv[k].w, lr, b1, b2, eps, inv_c1, inv_c2);
                const int64_t e = plane0 + (int64_t)(c0 + k) * HW;
                *reinterpret_cast<float4*>(p + e) = pp[k];
                *reinterpret_cast<float4*>(m + e) = mm[k];
                *reinterpret_cast<float4*>(v + e) = vv[k];
            }
        };
        int32_t c = 0;
        for (; c + CG <= C; c += CG) group(c, CG);
        if (c < C) group(c, C - c);
    } else {
        for (int32_t c = 0; c < C; c++) {
            const int64_t e = plane0 + (int64_t)c * HW;
            float pp = p[e], mm = m[e], vv = v[e];
            adam_elem(pp, g[e], mm, vv, lr, b1, b2, eps, inv_c1, inv_c2);
            p[e] = pp;
            m[e] = mm;
            v[e] = vv;
        }
    }
}

__global__ void k_step_inc(int32_t* step) { *step += 1; }

}  // namespace

hipError_t launch_loss_l1(const float* img, const float* tgt, int64_t n, float* g, double* partial, float* loss,
                          hipStream_t s) {
    const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                       reinterpret_cast<uintptr_t>(g)) & 15) == 0;
    if (vec) k_l1<true><<<kLossBlocks, 256, 0, s>>>(img, tgt, n, g, partial);
    else k_l1<false><<<kLossBlocks, 256, 0, s>>>(img, tgt, n, g, partial);
    k_l1_final<<<1, kLossBlocks, 0, s>>>(partial, n, loss);
    return hipGetLastError();
}

hipError_t launch_loss_l1_tiles(const double* tile_loss, int64_t n_tiles, int64_t n, float* loss, hipStream_t s) {
    k_l1_tiles<<<1, kLossBlocks, 0, s>>>(tile_loss, n_tiles, n, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* atlas, const float* grad, float* m, float* v, const uint8_t* visible,
                       const int32_t* texel_gauss, int64_t n_gauss, int32_t F, int32_t C, int32_t H, int32_t W,
                       float lr, float b1, float b2, float eps, int32_t step, int32_t* step_dev, hipStream_t s) {
    const int64_t HW = (int64_t)H * W;
    if (step_dev) k_step_inc<<<1, 1, 0, s>>>(step_dev);
    if (HW == 0) return hipGetLastError();
    const double c1 = step_dev ? 1.0 : 1.0 - pow((double)b1, (double)step);
    const double c2 = step_dev ? 1.0 : 1.0 - pow((double)b2, (double)step);
    const bool vec = HW % 4 == 0 && ((reinterpret_cast<uintptr_t>(atlas) | reinterpret_cast<uintptr_t>(grad) |
                                      reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
    const int64_t threads = vec ? HW / 4 : HW;
    const dim3 grid((unsigned)ceil_div(threads, 256), (unsigned)F);
    if (vec)
        k_adam<true><<<grid, 256, 0, s>>>(atlas, grad, m, v, visible, texel_gauss, n_gauss, C, HW, lr, b1, b2, eps,
                                          (float)(1.0 / c1), (float)(1.0 / c2), step_dev);
    else
        k_adam<false><<<grid, 256, 0, s>>>(atlas, grad, m, v, visible, texel_gauss, n_gauss, C, HW, lr, b1, b2, eps,
                                           (float)(1.0 / c1), (float)(1.0 / c2), step_dev);
    return hipGetLastError();
}

}  // namespace pg
