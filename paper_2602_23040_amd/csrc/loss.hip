// Objective terms of Sec. 4.2 "Objective": the photometric blend and the
// scale / opacity regularisers.
//
// Photometric objective:
//   L = (1 - lambda) mean |I - T| + lambda (1 - mean SSIM(I, T))
// over every view, pixel and channel, and its cotangent dL/dI, in one pass.
//
// SSIM per channel plane: local statistics under an 11 x 11 Gaussian window
// (sigma 1.5, weights summing to 1) with zero padding outside the view,
//   S = (2 a b + C1) (2 s_xy + C2) / ((a^2 + b^2 + C1) (s_x + s_y + C2)),
// a, b the window means, s_x, s_y, s_xy the window (co)variances,
// C1 = 0.01^2, C2 = 0.03^2.  Its gradient with respect to the image is the
// window correlation (the window is symmetric, so its own adjoint) of the
// partials P_a = dS/da, P_c = dS/dE[x^2], P_e = dS/dE[xy]:
//   dS/dx_q = (w * P_a)_q + 2 x_q (w * P_c)_q + y_q (w * P_e)_q.
//
// One work-group of 512 threads per 32 x 32 pixel block of a view and one
// channel at a time (the next channel's inputs load while one is computed).  Everything stays in LDS: the inputs with a 10-pixel
// halo, their separable window sums over the 42 x 42 region the adjoint
// needs, the three partial maps there (zero outside the view, where no S is
// taken), and their separable blur back to the block.  The inputs are
// shifted by the block's first pixel before squaring (E[x~^2] - a~^2 with
// x~ = x - k equals the variance, padding included, since the window sums to
// 1), which keeps FP32 cancellation in the variances small.  Per-block sums
// of S and |I - T| (FP64) go to a small partial array that k_photo_final
// reduces.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kR = 5;                       // window half-width
constexpr int kK = 2 * kR + 1;
constexpr int kB = 32;                      // output block side
constexpr int kIW = kB + 4 * kR;            // input patch side (42 + 10 = 52 with 2 halos)
constexpr int kMW = kB + 2 * kR;            // partial-map region side (42)
constexpr int kThreads = 512;              // two output pixels per thread in the last pass
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Win {
    float w[kK];
};

__device__ __forceinline__ double block_sum_d(double v, double* s_w) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kThreads / 64; k++) t += s_w[k];
    return t;
}

// blocks: one per 32 x 32 block of every view, numbered per view row-major
// (ceil(W/32) x ceil(H/32)) from blk_base[v].
__global__ __launch_bounds__(kThreads) void k_photo(const ViewDev* __restrict__ views, int nv,
                                                    const int64_t* __restrict__ blk_base,
                                                    const float* __restrict__ image, const float* __restrict__ target,
                                                    Win win, float lambda, double inv_n, float* __restrict__ dimg,
                                                    double* __restrict__ partial) {
    // LDS by lifetime: the input patch, then (over it) the partial maps; the
    // window sums, then (over them) the adjoint's horizontal blur.  65 KB, so
    // two work-groups share a CU.
    __shared__ float s_in[2 * kIW * kIW];
    __shared__ float s_h5[5 * kIW * kMW];
    __shared__ double s_w[kThreads / 64];
    static_assert(3 * kMW * kMW <= 2 * kIW * kIW && 3 * kMW * kB <= 5 * kIW * kMW, "LDS aliasing");
    float* sx = s_in;
    float* sy = s_in + kIW * kIW;
    float (*h5)[kIW * kMW] = reinterpret_cast<float (*)[kIW * kMW]>(s_h5);
    float (*sm)[kMW * kMW] = reinterpret_cast<float (*)[kMW * kMW]>(s_in);
    float (*h3)[kMW * kB] = reinterpret_cast<float (*)[kMW * kB]>(s_h5);
    // view of this block (binary search over the per-view block bases)
    const int64_t blk = blockIdx.x;
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_base[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    const ViewDev& V = views[lo];
    const int32_t BX = (V.W + kB - 1) / kB;
    const int64_t local = blk - blk_base[lo];
    const int32_t x0 = (int32_t)(local % BX) * kB, y0 = (int32_t)(local / BX) * kB;
    const int64_t HW = (int64_t)V.W * V.H;
    const int t = threadIdx.x;
    double s_sum = 0.0, l1_sum = 0.0;
    // each thread's share of a channel's input patch, loaded one channel ahead
    constexpr int kPer = (kIW * kIW + kThreads - 1) / kThreads;
    float px[kPer], py[kPer];
    auto fetch = [&](int ch) __attribute__((always_inline)) {
        const float* X = image + 3 * V.pix_base + ch * HW;
        const float* Y = target + 3 * V.pix_base + ch * HW;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int k = t + u * kThreads;
            const int gx = x0 - 2 * kR + k % kIW, gy = y0 - 2 * kR + k / kIW;
            const bool in = k < kIW * kIW && gx >= 0 && gx < V.W && gy >= 0 && gy < V.H;
            const int64_t p = (int64_t)gy * V.W + gx;
            px[u] = in ? X[p] : 0.0f;
            py[u] = in ? Y[p] : 0.0f;
        }
    };
    fetch(0);
    for (int ch = 0; ch < 3; ch++) {
        const float* X = image + 3 * V.pix_base + ch * HW;
        const float* Y = target + 3 * V.pix_base + ch * HW;
        const float kx = X[(int64_t)y0 * V.W + x0], ky = Y[(int64_t)y0 * V.W + x0];
        __syncthreads();   // the previous channel is done with the LDS
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int k = t + u * kThreads;
            if (k < kIW * kIW) {
                sx[k] = px[u] - kx;
                sy[k] = py[u] - ky;
            }
        }
        __syncthreads();
        if (ch < 2) fetch(ch + 1);   // in flight while this channel is computed
        // horizontal window sums: input rows x partial-map columns, two adjacent
        // columns per item (12 loads per input plane for 22 taps)
        for (int k = t; k < kIW * (kMW / 2); k += kThreads) {
            const int r = k / (kMW / 2), c = 2 * (k % (kMW / 2));
            float a0 = 0.f, b0 = 0.f, c0 = 0.f, d0 = 0.f, e0 = 0.f;
            float a1 = 0.f, b1 = 0.f, c1 = 0.f, d1 = 0.f, e1 = 0.f;
            float xp = sx[r * kIW + c], yp = sy[r * kIW + c];
#pragma unroll
            for (int j = 0; j < kK; j++) {
                const float xn = sx[r * kIW + c + j + 1], yn = sy[r * kIW + c + j + 1], w = win.w[j];
                a0 = fmaf(w, xp, a0);
                b0 = fmaf(w, yp, b0);
                c0 = fmaf(w, xp * xp, c0);
                d0 = fmaf(w, yp * yp, d0);
                e0 = fmaf(w, xp * yp, e0);
                a1 = fmaf(w, xn, a1);
                b1 = fmaf(w, yn, b1);
                c1 = fmaf(w, xn * xn, c1);
                d1 = fmaf(w, yn * yn, d1);
                e1 = fmaf(w, xn * yn, e1);
                xp = xn;
                yp = yn;
            }
            const int o = r * kMW + c;
            h5[0][o] = a0;
            h5[1][o] = b0;
            h5[2][o] = c0;
            h5[3][o] = d0;
            h5[4][o] = e0;
            h5[0][o + 1] = a1;
            h5[1][o + 1] = b1;
            h5[2][o + 1] = c1;
            h5[3][o + 1] = d1;
            h5[4][o + 1] = e1;
        }
        __syncthreads();
        // vertical window sums on the partial-map region -> S and its partials,
        // two adjacent rows per item
        for (int k = t; k < (kMW / 2) * kMW; k += kThreads) {
            const int r0 = 2 * (k / kMW), c = k % kMW;
            float m0[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, m1[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            float prev[5];
#pragma unroll
            for (int q = 0; q < 5; q++) prev[q] = h5[q][r0 * kMW + c];
#pragma unroll
            for (int j = 0; j < kK; j++) {
                const float w = win.w[j];
#pragma unroll
                for (int q = 0; q < 5; q++) {
                    const float nx = h5[q][(r0 + j + 1) * kMW + c];
                    m0[q] = fmaf(w, prev[q], m0[q]);
                    m1[q] = fmaf(w, nx, m1[q]);
                    prev[q] = nx;
                }
            }
#pragma unroll
            for (int half = 0; half < 2; half++) {
                const float* m = half ? m1 : m0;
                const int r = r0 + half;
                const int gx = x0 - kR + c, gy = y0 - kR + r;
                float pa = 0.f, pc = 0.f, pe = 0.f;
                if (gx >= 0 && gx < V.W && gy >= 0 && gy < V.H) {
                    const float a = m[0] + kx, b = m[1] + ky;
                    const float vx = m[2] - m[0] * m[0], vy = m[3] - m[1] * m[1], cxy = m[4] - m[0] * m[1];
                    const float N1 = 2.0f * a * b + kC1, N2 = 2.0f * cxy + kC2;
                    const float D1 = a * a + b * b + kC1, D2 = vx + vy + kC2;
                    const float iD = 1.0f / (D1 * D2);
                    const float S = N1 * N2 * iD;
                    pa = 2.0f * b * (N2 - N1) * iD - S * (2.0f * a / D1 - 2.0f * a / D2);
                    pc = -S / D2;
                    pe = 2.0f * N1 * iD;
                    if (r >= kR && r < kR + kB && c >= kR && c < kR + kB) s_sum += (double)S;
                }
                sm[0][r * kMW + c] = pa;
                sm[1][r * kMW + c] = pc;
                sm[2][r * kMW + c] = pe;
            }
        }
        __syncthreads();
        // adjoint: blur the partial maps back to the block (horizontal, then
        // vertical), two adjacent columns per item
        for (int k = t; k < kMW * (kB / 2); k += kThreads) {
            const int r = k / (kB / 2), c = 2 * (k % (kB / 2));
            float a0 = 0.f, c0 = 0.f, e0 = 0.f, a1 = 0.f, c1 = 0.f, e1 = 0.f;
            float pa = sm[0][r * kMW + c], pc = sm[1][r * kMW + c], pe = sm[2][r * kMW + c];
#pragma unroll
            for (int j = 0; j < kK; j++) {
                const float w = win.w[j];
                const int o = r * kMW + c + j + 1;
                const float na = sm[0][o], nc = sm[1][o], ne = sm[2][o];
                a0 = fmaf(w, pa, a0);
                c0 = fmaf(w, pc, c0);
                e0 = fmaf(w, pe, e0);
                a1 = fmaf(w, na, a1);
                c1 = fmaf(w, nc, c1);
                e1 = fmaf(w, ne, e1);
                pa = na;
                pc = nc;
                pe = ne;
            }
            const int o = r * kB + c;
            h3[0][o] = a0;
            h3[1][o] = c0;
            h3[2][o] = e0;
            h3[0][o + 1] = a1;
            h3[1][o + 1] = c1;
            h3[2][o + 1] = e1;
        }
        __syncthreads();
        for (int o = t; o < kB * kB; o += kThreads) {
            const int tx = o % kB, ty = o / kB;
            float ga = 0.f, gc = 0.f, ge = 0.f;
#pragma unroll
            for (int j = 0; j < kK; j++) {
                const float w = win.w[j];
                ga = fmaf(w, h3[0][(ty + j) * kB + tx], ga);
                gc = fmaf(w, h3[1][(ty + j) * kB + tx], gc);
                ge = fmaf(w, h3[2][(ty + j) * kB + tx], ge);
            }
            const int gx = x0 + tx, gy = y0 + ty;
            if (gx < V.W && gy < V.H) {
                const int64_t p = (int64_t)gy * V.W + gx;
                const float xv = X[p], yv = Y[p];
                const float gs = ga + 2.0f * xv * gc + yv * ge;
                const float df = xv - yv;
                const float sg = df > 0.f ? 1.f : (df < 0.f ? -1.f : 0.f);
                dimg[3 * V.pix_base + ch * HW + p] =
                    (float)(((double)(1.0f - lambda) * sg - (double)lambda * gs) * inv_n);
                l1_sum += (double)fabsf(df);
            }
        }
    }
    const double ts = block_sum_d(s_sum, s_w);
    const double tl = block_sum_d(l1_sum, s_w);
    if (t == 0) {
        partial[2 * blk] = ts;
        partial[2 * blk + 1] = tl;
    }
}

__global__ __launch_bounds__(1024) void k_photo_final(const double* __restrict__ partial, int64_t n_blk,
                                                      float lambda, double inv_n, float* __restrict__ loss) {
    __shared__ double s_s[16], s_l[16];
    double ss = 0.0, sl = 0.0;
    for (int64_t i = threadIdx.x; i < n_blk; i += 1024) {
        ss += partial[2 * i];
        sl += partial[2 * i + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ss += __shfl_xor(ss, o, 64);
        sl += __shfl_xor(sl, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_s[threadIdx.x >> 6] = ss;
        s_l[threadIdx.x >> 6] = sl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ss = 0.0;
        sl = 0.0;
        for (int k = 0; k < 16; k++) {
            ss += s_s[k];
            sl += s_l[k];
        }
        *loss = (float)((1.0 - (double)lambda) * sl * inv_n + (double)lambda * (1.0 - ss * inv_n));
    }
}

// ---------------------------------------------------------------- regularisers
// Scale and opacity regularisers of the objective over the Gaussians of every
// frame (or the dynamic ones):  L_scale = mean max(0, max_k s_k - s_max)^2,
// L_opacity = mean o (1 - o), s = exp(l_s), o = sigmoid(l_o), in FP64 from
// the FP32 texel values.  Three kernels: block sums of (count, hinge^2,
// o (1 - o)); their total and the two means; the weighted gradients added to
// the texel gradient (l_s through exp on the largest scale's channel, l_o
// through the sigmoid), divided by the count.
constexpr int kRegThreads = 256;

struct RegTerms {
    int kmax;
    double smax, h, o;
};

__device__ __forceinline__ RegTerms reg_terms(const float* P, int64_t stride, double s_max) {
    RegTerms r;
    r.kmax = 0;
    r.smax = exp((double)P[3 * stride]);
    for (int k = 1; k < 3; k++) {
        const double sk = exp((double)P[(3 + k) * stride]);
        if (sk > r.smax) {
            r.smax = sk;
            r.kmax = k;
        }
    }
    r.h = r.smax > s_max ? r.smax - s_max : 0.0;
    r.o = 1.0 / (1.0 + exp(-(double)P[10 * stride]));
    return r;
}

__global__ __launch_bounds__(kRegThreads) void k_reg_sum(const float* __restrict__ params,
                                                         const int64_t* __restrict__ n_dev, int64_t n_cap,
                                                         int32_t F, int32_t C, const uint8_t* __restrict__ dyn,
                                                         double s_max, double* __restrict__ partial) {
    __shared__ double s_w[3][kRegThreads / 64];
    const int64_t n = imin(*n_dev, n_cap);
    double cnt = 0.0, hs = 0.0, os = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * kRegThreads + threadIdx.x; g < (int64_t)F * n;
         g += (int64_t)gridDim.x * kRegThreads) {
        const int32_t f = (int32_t)(g / n);
        const int64_t i = g - (int64_t)f * n;
        if (dyn && !dyn[(int64_t)f * n_cap + i]) continue;
        const RegTerms r = reg_terms(params + (int64_t)f * C * n_cap + i, n_cap, s_max);
        cnt += 1.0;
        hs += r.h * r.h;
        os += r.o * (1.0 - r.o);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        hs += __shfl_xor(hs, o, 64);
        os += __shfl_xor(os, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_w[0][threadIdx.x >> 6] = cnt;
        s_w[1][threadIdx.x >> 6] = hs;
        s_w[2][threadIdx.x >> 6] = os;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < kRegThreads / 64; w++) t += s_w[threadIdx.x][w];
        partial[3 * blockIdx.x + threadIdx.x] = t;
    }
}

// partial[3 PG_REG_BLOCKS] <- the count; loss[0..1] <- the two means
__global__ void k_reg_final(double* __restrict__ partial, float* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double cnt = 0.0, hs = 0.0, os = 0.0;
    for (int b = 0; b < PG_REG_BLOCKS; b++) {
        cnt += partial[3 * b];
        hs += partial[3 * b + 1];
        os += partial[3 * b + 2];
    }
    partial[3 * PG_REG_BLOCKS] = cnt;
    loss[0] = cnt > 0.0 ? (float)(hs / cnt) : 0.0f;
    loss[1] = cnt > 0.0 ? (float)(os / cnt) : 0.0f;
}

__global__ __launch_bounds__(kRegThreads) void k_reg_grad(const float* __restrict__ params,
                                                          const int64_t* __restrict__ n_dev, int64_t n_cap,
                                                          int32_t F, int32_t C, const uint8_t* __restrict__ dyn,
                                                          const int32_t* __restrict__ gauss_texel, int64_t HW,
                                                          double s_max, double w_scale, double w_opacity,
                                                          const double* __restrict__ partial,
                                                          float* __restrict__ gatlas) {
    const int64_t n = imin(*n_dev, n_cap);
    const double cnt = partial[3 * PG_REG_BLOCKS];
    const int64_t g = (int64_t)blockIdx.x * kRegThreads + threadIdx.x;
    if (g >= (int64_t)F * n || cnt <= 0.0) return;
    const int32_t f = (int32_t)(g / n);
    const int64_t i = g - (int64_t)f * n;
    if (dyn && !dyn[(int64_t)f * n_cap + i]) return;
    const RegTerms r = reg_terms(params + (int64_t)f * C * n_cap + i, n_cap, s_max);
    float* out = gatlas + (int64_t)f * C * HW + gauss_texel[i];
    if (r.h > 0.0) out[(int64_t)(3 + r.kmax) * HW] += (float)(w_scale * (2.0 * r.h * r.smax) / cnt);
    out[10 * HW] += (float)(w_opacity * ((1.0 - 2.0 * r.o) * r.o * (1.0 - r.o)) / cnt);
}

}  // namespace

hipError_t launch_regularisers(const float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C,
                               const int32_t* gauss_texel, int64_t HW, const uint8_t* dyn, double s_max,
                               double w_scale, double w_opacity, float* gatlas, float* loss, double* partial,
                               hipStream_t s) {
    k_reg_sum<<<PG_REG_BLOCKS, kRegThreads, 0, s>>>(params, n_dev, n_cap, F, C, dyn, s_max, partial);
    k_reg_final<<<1, 64, 0, s>>>(partial, loss);
    if (n_cap > 0)
        k_reg_grad<<<(unsigned)ceil_div((int64_t)F * n_cap, kRegThreads), kRegThreads, 0, s>>>(
            params, n_dev, n_cap, F, C, dyn, gauss_texel, HW, s_max, w_scale, w_opacity, partial, gatlas);
    return hipGetLastError();
}

int64_t photo_blocks(const pg_views* v) { return v->n_ssim_blocks; }

hipError_t launch_photo(const pg_views* v, const float* image, const float* target, float lambda, float* dimg,
                        float* loss, double* partial, hipStream_t s) {
    const int64_t nb = v->n_ssim_blocks;
    if (nb == 0 || v->n_pixels == 0) return hipSuccess;
    Win win;
    double g[kK], sum = 0.0;
    for (int k = 0; k < kK; k++) {
        const double d = (double)(k - kR);
        g[k] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < kK; k++) win.w[k] = (float)(g[k] / sum);
    const double inv_n = 1.0 / (3.0 * (double)v->n_pixels);
    k_photo<<<(unsigned)nb, kThreads, 0, s>>>(v->d_views, v->n_views, v->d_ssim_base, image, target, win, lambda,
                                              inv_n, dimg, partial);
    k_photo_final<<<1, 1024, 0, s>>>(partial, nb, lambda, inv_n, loss);
    return hipGetLastError();
}

}  // namespace pg
