// a2 -- EWA projection of every Gaussian into every view of its frame, and
// (a5, second half) its adjoint back to the texel channels.
//
// Formulas: Sigma = R(q) diag(s)^2 R(q)^T; Sigma_c = W Sigma W^T; J the
// perspective Jacobian at the camera-space mean; Sigma2D = J Sigma_c J^T
// with +0.3 added to the diagonal; det / z validity test; lambda_max and the
// radius ceil(3 sqrt(lambda_max)) ("Covariance-Aware Gaussian Masking",
// Sec. 4.2, and Algorithm 1 steps 1-4); X_c = R X + t and the pixel mean
// (supplementary, viewer section); SH colour of the 3DGS record (Sec. 3).
//
// Every quantity that decides an integer (culls, radius, tile rectangle,
// depth key) is computed in FP64 from the FP32 texels in one fixed order:
// sums of products left to right in ascending index, no contraction (this
// file is compiled with -ffp-contract=off), IEEE division and square root.
// The outputs the compositing kernels read are rounded to FP32 once.
//
// Launch shape: one thread per Gaussian of a frame; the thread reads the
// texel record once and loops over the views of that frame, so a batched
// call reads the parameters once instead of once per view.  Work per
// (Gaussian, view) is ~300 FP64 flops against 64 bytes written, so at the
// chip's FP64 rate the kernel stays close to its HBM bound.
//
// The adjoint runs as three passes: a streaming sum of each record's
// instance slots, the geometric chain in FP64 (position, scale, rotation,
// opacity), and the SH colour chain in FP32 (its 48 coefficient gradients and
// the view-direction term of the position gradient).  Splitting them keeps
// both under 256 registers without spills.
#include "pg_internal.h"

#pragma clang fp contract(off)

namespace pg {

namespace {

constexpr double kNearZ = 0.2;
constexpr double kLowPass = 0.3;
constexpr double kDetMin = 1e-7;

// Real SH normalisations (Condon-Shortley phase kept).
constexpr double kY0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15 / pi) / 2
constexpr double kY2b = 0.31539156525252005;  // sqrt(5 / pi) / 4
constexpr double kY2c = 0.5462742152960396;   // sqrt(15 / pi) / 4
constexpr double kY3a = 0.5900435899266435;   // sqrt(35 / (2 pi)) / 4
constexpr double kY3b = 2.890611442640554;    // sqrt(105 / pi) / 2
constexpr double kY3c = 0.4570457994644658;   // sqrt(21 / (2 pi)) / 4
constexpr double kY3d = 0.3731763325901154;   // sqrt(7 / pi) / 4
constexpr double kY3e = 1.445305721320277;    // sqrt(105 / pi) / 4

template <int L>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double* Y) {
    Y[0] = kY0;
    if (L >= 1) {
        Y[1] = -kY1 * y;
        Y[2] = kY1 * z;
        Y[3] = -kY1 * x;
    }
    if (L >= 2) {
        Y[4] = kY2a * x * y;
        Y[5] = -kY2a * y * z;
        Y[6] = kY2b * (3.0 * z * z - 1.0);
        Y[7] = -kY2a * x * z;
        Y[8] = kY2c * (x * x - y * y);
    }
    if (L >= 3) {
        Y[9] = -kY3a * y * (3.0 * x * x - y * y);
        Y[10] = kY3b * x * y * z;
        Y[11] = -kY3c * y * (5.0 * z * z - 1.0);
        Y[12] = kY3d * z * (5.0 * z * z - 3.0);
        Y[13] = -kY3c * x * (5.0 * z * z - 1.0);
        Y[14] = kY3e * z * (x * x - y * y);
        Y[15] = -kY3a * x * (x * x - 3.0 * y * y);
    }
}

// World-space part of the chain, shared by every view of a Gaussian.
struct World {
    double mu[3], s[3], qn, qh[4], o;
    double Rq[9], M[9], S[9];
};

__device__ __forceinline__ void world_chain(const float* rec, World& w) {
    w.mu[0] = rec[0]; w.mu[1] = rec[1]; w.mu[2] = rec[2];
    w.s[0] = exp((double)rec[3]); w.s[1] = exp((double)rec[4]); w.s[2] = exp((double)rec[5]);
    const double qw = rec[6], qx = rec[7], qy = rec[8], qz = rec[9];
    w.qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    w.qh[0] = qw / w.qn; w.qh[1] = qx / w.qn; w.qh[2] = qy / w.qn; w.qh[3] = qz / w.qn;
    w.o = 1.0 / (1.0 + exp(-(double)rec[10]));
    const double a = w.qh[0], x = w.qh[1], y = w.qh[2], z = w.qh[3];
    w.Rq[0] = 1.0 - 2.0 * (y * y + z * z);
    w.Rq[1] = 2.0 * (x * y - a * z);
    w.Rq[2] = 2.0 * (x * z + a * y);
    w.Rq[3] = 2.0 * (x * y + a * z);
    w.Rq[4] = 1.0 - 2.0 * (x * x + z * z);
    w.Rq[5] = 2.0 * (y * z - a * x);
    w.Rq[6] = 2.0 * (x * z - a * y);
    w.Rq[7] = 2.0 * (y * z + a * x);
    w.Rq[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) w.M[3 * r + k] = w.Rq[3 * r + k] * w.s[k];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int k = 0; k < 3; k++)
            w.S[3 * r + k] = (w.M[3 * r] * w.M[3 * k] + w.M[3 * r + 1] * w.M[3 * k + 1]) + w.M[3 * r + 2] * w.M[3 * k + 2];
}

// Camera part of the chain.
struct Cam {
    double xc, yc, zc;
    double Sc[9], J[6];
    double ap, bp, cp, det;
};

__device__ __forceinline__ bool camera_chain(const ViewDev& V, const World& w, Cam& c) {
    const double* R = V.R;
    c.xc = ((R[0] * w.mu[0] + R[1] * w.mu[1]) + R[2] * w.mu[2]) + V.t[0];
    c.yc = ((R[3] * w.mu[0] + R[4] * w.mu[1]) + R[5] * w.mu[2]) + V.t[1];
    c.zc = ((R[6] * w.mu[0] + R[7] * w.mu[1]) + R[8] * w.mu[2]) + V.t[2];
    if (!(c.zc > kNearZ)) return false;
    double A[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) A[3 * r + k] = (R[3 * r] * w.S[k] + R[3 * r + 1] * w.S[3 + k]) + R[3 * r + 2] * w.S[6 + k];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) c.Sc[3 * r + k] = (A[3 * r] * R[3 * k] + A[3 * r + 1] * R[3 * k + 1]) + A[3 * r + 2] * R[3 * k + 2];
    const double z2 = c.zc * c.zc;
    c.J[0] = V.fx / c.zc;
    c.J[1] = 0.0;
    c.J[2] = -(V.fx * c.xc) / z2;
    c.J[3] = 0.0;
    c.J[4] = V.fy / c.zc;
    c.J[5] = -(V.fy * c.yc) / z2;
    double T[6];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) T[3 * r + k] = (c.J[3 * r] * c.Sc[k] + c.J[3 * r + 1] * c.Sc[3 + k]) + c.J[3 * r + 2] * c.Sc[6 + k];
    const double s00 = (T[0] * c.J[0] + T[1] * c.J[1]) + T[2] * c.J[2];
    const double s01 = (T[0] * c.J[3] + T[1] * c.J[4]) + T[2] * c.J[5];
    const double s11 = (T[3] * c.J[3] + T[4] * c.J[4]) + T[5] * c.J[5];
    c.ap = s00 + kLowPass;
    c.bp = s01;
    c.cp = s11 + kLowPass;
    c.det = c.ap * c.cp - c.bp * c.bp;
    return true;
}

template <int L>
__device__ __forceinline__ void view_dir(const ViewDev& V, const World& w, double d[3], double* dn) {
    d[0] = w.mu[0] - V.cw[0];
    d[1] = w.mu[1] - V.cw[1];
    d[2] = w.mu[2] - V.cw[2];
    *dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    const double inv = 1.0 / *dn;      // the direction only feeds the colour (no integer decision)
    d[0] *= inv; d[1] *= inv; d[2] *= inv;
}

// ---- FP32 SH basis and its contracted gradient for the colour adjoint

template <int L>
__device__ __forceinline__ void sh_basis_f(float x, float y, float z, float* Y) {
    Y[0] = (float)kY0;
    if (L >= 1) {
        Y[1] = -(float)kY1 * y;
        Y[2] = (float)kY1 * z;
        Y[3] = -(float)kY1 * x;
    }
    if (L >= 2) {
        Y[4] = (float)kY2a * x * y;
        Y[5] = -(float)kY2a * y * z;
        Y[6] = (float)kY2b * (3.0f * z * z - 1.0f);
        Y[7] = -(float)kY2a * x * z;
        Y[8] = (float)kY2c * (x * x - y * y);
    }
    if (L >= 3) {
        Y[9] = -(float)kY3a * y * (3.0f * x * x - y * y);
        Y[10] = (float)kY3b * x * y * z;
        Y[11] = -(float)kY3c * y * (5.0f * z * z - 1.0f);
        Y[12] = (float)kY3d * z * (5.0f * z * z - 3.0f);
        Y[13] = -(float)kY3c * x * (5.0f * z * z - 1.0f);
        Y[14] = (float)kY3e * z * (x * x - y * y);
        Y[15] = -(float)kY3a * x * (x * x - 3.0f * y * y);
    }
}

template <int L>
__device__ __forceinline__ void sh_grad_dot_f(float x, float y, float z, const float* w, float g[3]) {
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    if (L >= 1) {
        g0 -= (float)kY1 * w[3];
        g1 -= (float)kY1 * w[1];
        g2 += (float)kY1 * w[2];
    }
    if (L >= 2) {
        g0 += (float)kY2a * y * w[4] - (float)kY2a * z * w[7] + 2.0f * (float)kY2c * x * w[8];
        g1 += (float)kY2a * x * w[4] - (float)kY2a * z * w[5] - 2.0f * (float)kY2c * y * w[8];
        g2 += -(float)kY2a * y * w[5] + 6.0f * (float)kY2b * z * w[6] - (float)kY2a * x * w[7];
    }
    if (L >= 3) {
        const float p3 = 3.0f * x * x - 3.0f * y * y, p5 = 5.0f * z * z - 1.0f;
        g0 += -6.0f * (float)kY3a * x * y * w[9] + (float)kY3b * y * z * w[10] - (float)kY3c * p5 * w[13] + 2.0f * (float)kY3e * x * z * w[14]
              - (float)kY3a * p3 * w[15];
        g1 += -(float)kY3a * p3 * w[9] + (float)kY3b * x * z * w[10] - (float)kY3c * p5 * w[11] - 2.0f * (float)kY3e * y * z * w[14]
              + 6.0f * (float)kY3a * x * y * w[15];
        g2 += (float)kY3b * x * y * w[10] - 10.0f * (float)kY3c * y * z * w[11] + (float)kY3d * (15.0f * z * z - 3.0f) * w[12]
              - 10.0f * (float)kY3c * x * z * w[13] + (float)kY3e * (x * x - y * y) * w[14];
    }
    g[0] = g0;
    g[1] = g1;
    g[2] = g2;
}

// Tile culling by the ellipse.  A tile of the rectangle is kept when the
// smallest q over the rectangle spanned by its pixel centres is at most 9 +
// 1e-3 (the margin covers the compositor's FP32 evaluation of q): zero when
// the mean lies inside, else the least of the four edge minima, each the
// parabola on that edge at its clamped vertex (on x = X the vertex is at
// y = (-B / C) X, on y = Y at x = (-B / A) Y).  Rectangles of more than
// kMaskTiles tiles keep every tile.  This is an optimisation of the method's
// tile lists (every tile of the rectangle): a dropped tile has q > 9 at every
// pixel centre, so no pixel of it would composite the Gaussian, and the image
// and gradients do not change.
constexpr int kMaskTiles = 64;
constexpr double kQCull = 9.001;
constexpr int kProjBlk = 128;

__device__ __forceinline__ double q_at(double A, double B, double C, double X, double Y) {
    return (A * X * X + 2.0 * B * X * Y) + C * Y * Y;
}

// Least q over the pixel-centre rectangle [X0, X1] x [Y0, Y1] (offsets from the mean).
__device__ __forceinline__ double rect_qmin(double A, double B, double C, double ky, double kx, double X0,
                                            double X1, double Y0, double Y1) {
    if (X0 <= 0.0 && X1 >= 0.0 && Y0 <= 0.0 && Y1 >= 0.0) return 0.0;
    const double ya = fmin(fmax(ky * X0, Y0), Y1), yb = fmin(fmax(ky * X1, Y0), Y1);
    const double xa = fmin(fmax(kx * Y0, X0), X1), xb = fmin(fmax(kx * Y1, X0), X1);
    return fmin(fmin(q_at(A, B, C, X0, ya), q_at(A, B, C, X1, yb)),
                fmin(q_at(A, B, C, xa, Y0), q_at(A, B, C, xb, Y1)));
}

// One thread per Gaussian, looping over the views of its frame.  The loop
// runs the work-group's largest view count on every thread (threads past
// their own count only take part in the tile tests), because each view's
// tile tests are shared out over the work-group: rectangles range from one
// tile to dozens, so a thread testing only its own would hold its wave for
// the largest rectangle among 64.  Per view: every thread stages its record
// (mean, conic, edge-vertex slopes, rectangle) in LDS; a work-group scan of
// the rectangles' tile counts numbers the (record, tile) tests, and each
// record writes its tests' (owner, tile) words at its place in that
// numbering; thread t takes tests t, t + 128, ... and ORs kept tiles into
// the owner's LDS mask.
template <int L>
__global__ __launch_bounds__(kProjBlk) void k_project(const ViewDev* __restrict__ views,
                                                      const int32_t* __restrict__ frame_views,
                                                      const int32_t* __restrict__ view_order, int32_t F, int32_t C,
                                                      int64_t N, int32_t tw, int32_t th,
                                                      const float* __restrict__ params,
                                                      pg_splat* __restrict__ splats, pg_bin* __restrict__ bins,
                                                      pg_tile_set* __restrict__ tiles,
                                                      uint8_t* __restrict__ visible) {
    constexpr int NB = (L + 1) * (L + 1);
    __shared__ double s_geo[7][kProjBlk];       // mean x, y; conic A, B, C; slopes -B/C, -B/A
    __shared__ int32_t s_rect[4][kProjBlk];     // x_lo, y_lo, width, 2^16 / width rounded up
    __shared__ uint16_t s_item[kProjBlk * kMaskTiles];   // test q: owner thread << 6 | rectangle bit
    __shared__ unsigned long long s_mask[kProjBlk];
    __shared__ int32_t s_wsum[kProjBlk / 64];
    const int tid = threadIdx.x;
    // grid (Gaussian chunks, frames): the frame, its views and so every view's camera
    // are uniform over the work-group, and the camera is read with scalar loads
    const int32_t f = (int32_t)blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * kProjBlk + tid;
    const bool in_range = i0 < N;
    const int64_t i = in_range ? i0 : 0;
    const int64_t g = (int64_t)f * N + i;
    const int32_t v0 = frame_views[f], v1 = frame_views[f + 1];
    const int32_t nv = v1 - v0;
    if (nv <= 0) return;     // uniform over the work-group
    const float* P = params + (int64_t)f * C * N + i;
    const bool has = in_range;
    float rec[11];
#pragma unroll
    for (int k = 0; k < 11; k++) rec[k] = has ? P[(int64_t)k * N] : 0.0f;
    float sh[3 * NB];
#pragma unroll
    for (int k = 0; k < 3 * NB; k++) sh[k] = has ? P[(int64_t)(11 + k) * N] : 0.0f;
    World w;
    world_chain(rec, w);
    const double itw = 1.0 / (double)tw, ith = 1.0 / (double)th;   // exact: tw, th are 8, 16 or 32
    bool any = false;
    for (int32_t k = 0; k < nv; k++) {
        const bool act = has;
        const int32_t v = view_order[v0 + k];
        const ViewDev& V = views[v];
        Cam c;
        float4 o0 = make_float4(0.f, 0.f, 0.f, 0.f), o1 = o0, o2 = o0;
        uint4 bo = make_uint4(0u, 0u, 0u, 0u);
        int32_t nrect = 0;      // tiles of the rectangle (0: culled)
        double mx = 0.0, my = 0.0, A = 1.0, B = 0.0, Cq = 1.0;
        int32_t ixl = 0, iyl = 0, ixh = 0, iyh = 0;
        bool ok = act && camera_chain(V, w, c) && (c.det > kDetMin);
        if (ok) {
            const double tr = c.ap + c.cp;
            const double lam = 0.5 * (tr + sqrt(fmax(0.0, tr * tr - 4.0 * c.det)));
            const double rr = ceil(3.0 * sqrt(lam));
            mx = (V.fx * c.xc) / c.zc + V.cx;
            my = (V.fy * c.yc) / c.zc + V.cy;
            // visibility (the set sparse Adam updates): some pixel of the image lies
            // within r of the mean on both axes; independent of the tile shape and of
            // the tile culling below
            if (mx + rr >= 0.0 && mx - rr < (double)V.W && my + rr >= 0.0 && my - rr < (double)V.H) any = true;
            // the view table only admits tile sides of 8, 16 or 32: dividing by a power of
            // two is exactly multiplying by its reciprocal, so these equal the divisions
            const double xlo = fmax(0.0, floor((mx - rr) * itw));
            const double xhi = fmin((double)(V.TX - 1), floor((mx + rr) * itw));
            const double ylo = fmax(0.0, floor((my - rr) * ith));
            const double yhi = fmin((double)(V.TY - 1), floor((my + rr) * ith));
            const float zf = (float)c.zc;
            double d[3], dn;
            view_dir<L>(V, w, d, &dn);
            double Y[16];
            sh_basis<L>(d[0], d[1], d[2], Y);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < NB; j++) acc += Y[j] * (double)sh[3 * j + ch];
                const double raw = 0.5 + acc;
                col[ch] = (float)(raw > 0.0 ? raw : 0.0);
            }
            // the conic decides no integer by itself (the tile test below keeps a
            // margin), so one reciprocal serves its three entries
            const double idet = 1.0 / c.det;
            A = c.cp * idet;
            B = -c.bp * idet;
            Cq = c.ap * idet;
            const uint64_t bx = (uint64_t)__double_as_longlong(mx), by = (uint64_t)__double_as_longlong(my);
            o0 = make_float4(__uint_as_float((uint32_t)bx), __uint_as_float((uint32_t)(bx >> 32)),
                             __uint_as_float((uint32_t)by), __uint_as_float((uint32_t)(by >> 32)));   // the FP64 mean's bits
            o1 = make_float4((float)A, (float)B, (float)Cq, (float)w.o);
            o2 = make_float4(col[0], col[1], col[2], zf);
            if (xlo <= xhi && ylo <= yhi) {
                ixl = (int32_t)xlo;
                iyl = (int32_t)ylo;
                ixh = (int32_t)xhi;
                iyh = (int32_t)yhi;
                nrect = (ixh - ixl + 1) * (iyh - iyl + 1);
                bo.x = (uint32_t)(ixl & 0xffff) | ((uint32_t)(iyl & 0xffff) << 16);
                bo.y = (uint32_t)(ixh & 0xffff) | ((uint32_t)(iyh & 0xffff) << 16);
                bo.z = __float_as_uint(zf);
            }
        }
        // ---- tile tests, shared out over the work-group
        const int32_t ntest = nrect <= kMaskTiles ? nrect : 0;
        const int32_t wdt = ixh - ixl + 1;
        s_geo[0][tid] = mx;
        s_geo[1][tid] = my;
        s_geo[2][tid] = A;
        s_geo[3][tid] = B;
        s_geo[4][tid] = Cq;
        const double iac = 1.0 / (A * Cq);         // edge-vertex slopes -B / C and -B / A
        s_geo[5][tid] = -B * A * iac;
        s_geo[6][tid] = -B * Cq * iac;
        s_rect[0][tid] = ixl;
        s_rect[1][tid] = iyl;
        s_rect[2][tid] = wdt;
        s_rect[3][tid] = (65536 + wdt - 1) / wdt;
        s_mask[tid] = 0ull;
        int32_t incl = ntest;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(incl, o, 64);
            if ((tid & 63) >= o) incl += u;
        }
        if ((tid & 63) == 63) s_wsum[tid >> 6] = incl;
        __syncthreads();
        if (tid >= 64) incl += s_wsum[0];
        for (int32_t b = 0; b < ntest; b++) s_item[incl - ntest + b] = (uint16_t)((tid << 6) | b);
        const int32_t total = s_wsum[0] + s_wsum[1];
        __syncthreads();
        for (int32_t q = tid; q < total; q += kProjBlk) {
            const uint32_t it = s_item[q];
            const int32_t lo = (int32_t)(it >> 6);                 // owner
            const int32_t bit = (int32_t)(it & 63u);               // row-major index in the rectangle
            const int32_t row = (bit * s_rect[3][lo]) >> 16;        // bit / width (bit < 64)
            const int32_t tx = s_rect[0][lo] + (bit - row * s_rect[2][lo]), ty = s_rect[1][lo] + row;
            const double X0 = ((double)tx * tw + 0.5) - s_geo[0][lo], X1 = X0 + (double)(tw - 1);
            const double Y0 = ((double)ty * th + 0.5) - s_geo[1][lo], Y1 = Y0 + (double)(th - 1);
            const double qmin = rect_qmin(s_geo[2][lo], s_geo[3][lo], s_geo[4][lo], s_geo[5][lo], s_geo[6][lo], X0,
                                          X1, Y0, Y1);
            if (qmin <= kQCull) atomicOr(&s_mask[lo], 1ull << bit);
        }
        __syncthreads();
        const uint64_t tmask = ntest ? (uint64_t)s_mask[tid] : 0ull;
        const int32_t nt = ntest ? (int32_t)__popcll(tmask) : nrect;
        uint4 ts = make_uint4(0u, 0u, 0u, 0u);
        if (nt > 0) {
            bo.w = (uint32_t)nt;
            ts = make_uint4((uint32_t)tmask, (uint32_t)(tmask >> 32), bo.x,
                            (uint32_t)(ixh - ixl + 1) | ((uint32_t)(iyh - iyl + 1) << 16));
        } else {
            bo = make_uint4(0u, 0u, 0u, 0u);
        }
        if (act) {
            const int64_t gv = (int64_t)v * N + i;
            float4* sp = reinterpret_cast<float4*>(splats + gv);
            sp[0] = o0;
            sp[1] = o1;
            sp[2] = o2;
            reinterpret_cast<uint4*>(bins)[gv] = bo;
            reinterpret_cast<uint4*>(tiles)[gv] = ts;
        }
    }
    if (any && has) visible[g] = 1;
}

// ---------------------------------------------------------------- flow masking
// Covariance-aware flow masking (Sec. 4.2 masking paragraph, Algorithm 1):
// a Gaussian is dynamic when, in some view of its frame, a pixel whose centre
// is within r = ceil(3 sqrt(lambda_max)) of the mean on both axes and inside
// the image has q <= 9 and a non-zero flow mask (the OR across cameras).
//
// k_tile_motion marks the screen tiles holding any motion (one wave per
// tile).  k_flow_mask then runs one thread per (view, Gaussian) record: the
// projection chain, culls and radius of k_project; the record stops there
// unless a tile under its square has motion.  The square is then scanned by
// the whole wave: the wave takes its flagged records one by one and tests 64
// pixels per round, only in tiles that hold motion (elsewhere the mask is
// zero), the mask byte first and q <= 9 in FP64 at the pixel centre, so the
// label is exactly that of a scan of every pixel of the square.  (One thread
// walking its own rows left the other lanes of its wave idle and issued one
// dependent mask load per pixel: 2.6 ms against 1.2 ms on 50 views.)  A hit
// writes 1 to the Gaussian's zeroed label: every writer stores the same
// value, so the OR over views needs no atomics.
__global__ __launch_bounds__(64) void k_tile_motion(const ViewDev* __restrict__ views, int nv, int64_t n_tiles,
                                                    int32_t tw, int32_t th, const uint8_t* __restrict__ masks,
                                                    uint8_t* __restrict__ tmot) {
    const int64_t tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const ViewDev& V = views[find_view_by_tile(views, nv, tile)];
    const int64_t local = tile - V.tile_base;
    const int32_t ty = (int32_t)(local / V.TX), tx = (int32_t)(local - (int64_t)ty * V.TX);
    bool any = false;
    for (int32_t k = threadIdx.x; k < tw * th; k += 64) {
        const int32_t x = tx * tw + k % tw, y = ty * th + k / tw;
        if (x < V.W && y < V.H) any |= masks[V.pix_base + (int64_t)y * V.W + x] != 0;
    }
    const uint64_t b = __ballot(any);
    if (threadIdx.x == 0) tmot[tile] = b ? 1 : 0;
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(128) void k_flow_mask(const ViewDev* __restrict__ views, int32_t C, int64_t N,
                                                   int64_t n_gv, int32_t tw, int32_t th,
                                                   const float* __restrict__ params,
                                                   const uint8_t* __restrict__ masks,
                                                   const uint8_t* __restrict__ tmot, uint8_t* __restrict__ dyn_gauss,
                                                   unsigned long long* __restrict__ counters) {
    // work-group b takes records [c * 128, c * 128 + 128) of view b / chunks (c = b mod
    // chunks): the view, so its camera, is uniform over the work-group (scalar loads)
    const int64_t chunks = (N + 127) / 128;
    const int32_t v = (int32_t)((int64_t)blockIdx.x / chunks);
    const int64_t i = ((int64_t)blockIdx.x - (int64_t)v * chunks) * 128 + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    uint64_t tests = 0;
    // this thread's record: projection, clipped square and the motion-tile test
    bool any = false;
    int32_t ix0 = 0, ix1 = -1, iy0 = 0, iy1 = -1;
    int64_t out = 0;
    double mx = 0.0, my = 0.0, A = 1.0, B = 0.0, Cq = 1.0;
    if (i < N) {
        const ViewDev& V = views[v];
        out = (int64_t)V.frame * N + i;
        const float* P = params + (int64_t)V.frame * C * N + i;
        float rec[11];
#pragma unroll
        for (int k = 0; k < 11; k++) rec[k] = P[(int64_t)k * N];
        World w;
        world_chain(rec, w);
        Cam c;
        if (camera_chain(V, w, c) && c.det > kDetMin) {
            const double tr = c.ap + c.cp;
            const double lam = 0.5 * (tr + sqrt(fmax(0.0, tr * tr - 4.0 * c.det)));
            const double rr = ceil(3.0 * sqrt(lam));
            mx = (V.fx * c.xc) / c.zc + V.cx;
            my = (V.fy * c.yc) / c.zc + V.cy;
            const double x0 = fmax(0.0, ceil(mx - rr - 0.5)), x1 = fmin((double)(V.W - 1), floor(mx + rr - 0.5));
            const double y0 = fmax(0.0, ceil(my - rr - 0.5)), y1 = fmin((double)(V.H - 1), floor(my + rr - 0.5));
            if (x0 <= x1 && y0 <= y1) {
                ix0 = (int32_t)x0;
                ix1 = (int32_t)x1;
                iy0 = (int32_t)y0;
                iy1 = (int32_t)y1;
                for (int32_t ty = iy0 / th; ty <= iy1 / th && !any; ty++)
                    for (int32_t tx = ix0 / tw; tx <= ix1 / tw; tx++)
                        if (tmot[V.tile_base + (int64_t)ty * V.TX + tx]) {
                            any = true;
                            break;
                        }
            }
            if (any) {
                A = c.cp / c.det;
                B = -c.bp / c.det;
                Cq = c.ap / c.det;
            }
        }
    }
    // The wave scans its flagged records one after another, all lanes on one
    // record: per motion tile under the record's square, 64 pixels per round,
    // the mask byte first and q <= 9 (FP64, at the pixel centre) only where it
    // is set; a ballot ends the record at its first hit.  Every pixel centre
    // of the clipped square lies in one of these tiles or has a zero mask.
    uint64_t todo = __ballot(any);
    while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int32_t rv = v;
        const int32_t sx0 = __shfl(ix0, src, 64), sx1 = __shfl(ix1, src, 64);
        const int32_t sy0 = __shfl(iy0, src, 64), sy1 = __shfl(iy1, src, 64);
        const double smx = __shfl(mx, src, 64), smy = __shfl(my, src, 64);
        const double sA = __shfl(A, src, 64), sB = __shfl(B, src, 64), sC = __shfl(Cq, src, 64);
        const ViewDev& V = views[rv];
        const uint8_t* M = masks + V.pix_base;
        const int32_t per_tile = tw * th;
        bool found = false;
        for (int32_t ty = sy0 / th; ty <= sy1 / th && !found; ty++) {
            for (int32_t tx = sx0 / tw; tx <= sx1 / tw && !found; tx++) {
                if (!tmot[V.tile_base + (int64_t)ty * V.TX + tx]) continue;
                for (int32_t b = 0; b < per_tile && !found; b += 64) {
                    const int32_t p = b + lane;
                    const int32_t x = tx * tw + p % tw, y = ty * th + p / tw;
                    bool hit = false;
                    if (p < per_tile && x >= sx0 && x <= sx1 && y >= sy0 && y <= sy1 && M[(int64_t)y * V.W + x]) {
                        tests++;
                        hit = q_at(sA, sB, sC, ((double)x + 0.5) - smx, ((double)y + 0.5) - smy) <= 9.0;
                    }
                    found = __ballot(hit) != 0;
                }
            }
        }
        const int64_t sout = __shfl(out, src, 64);
        if (found && lane == 0) dyn_gauss[sout] = 1;
    }
    if (counters) {
        unsigned long long t = tests;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0 && t) atomicAdd(counters, t);
    }
}

// Texel form of the labels: 1 where the texel's Gaussian is dynamic in some frame.
__global__ __launch_bounds__(256) void k_dyn_texel(const uint8_t* __restrict__ dyn_gauss,
                                                   const int32_t* __restrict__ texel_gauss, int64_t HW, int32_t F,
                                                   int64_t N, uint8_t* __restrict__ dyn_texel) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= HW) return;
    const int32_t gi = texel_gauss[t];
    uint8_t d = 0;
    if (gi >= 0 && gi < N)
        for (int32_t f = 0; f < F; f++) d |= dyn_gauss[(int64_t)f * N + gi];
    dyn_texel[t] = d;
}

// ---------------------------------------------------------------- adjoint
//
// With Q the conic matrix and Gh = [[da, db/2], [db/2, dc]] (q = a dx^2 +
// 2 b dx dy + c dy^2): dL/dSigma2D = -Q Gh Q; dL/dSigma_c = J^T (.) J;
// dL/dJ = 2 (dL/dSigma2D) J Sigma_c; dL/dSigma = W^T (dL/dSigma_c) W;
// dL/dM = 2 (dL/dSigma) M with M = R(q) diag(s); the mean through J and
// through dJ/dmu_c; SH through the basis and the view direction.  Texel
// chain: l_s via s, the raw quaternion via the normalisation, l_o via o (1 - o).
// Geometric part of the adjoint, FP64: position, log-scale, quaternion and
// logit-opacity gradients through the EWA chain of every view of the
// Gaussian's frame.  FP64 because the gradient of a rotation about an
// elongated Gaussian's long axis (and the quaternion's tangent component in
// general) is a small difference of large terms: in FP32 a few texels of the
// 2048^2 workload missed 1e-3.  No SH coefficients are held here.
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_project_bwd_geo(const ViewDev* __restrict__ views,
                                                         const int32_t* __restrict__ frame_views,
                                                         const int32_t* __restrict__ view_order, int32_t F,
                                                         int32_t C, int64_t N, int64_t n_gv,
                                                         const float* __restrict__ params,
                                                         float* __restrict__ grad2d,
                                                         const int32_t* __restrict__ gauss_texel,
                                                         const uint8_t* __restrict__ dyn, int64_t HW,
                                                         float* __restrict__ gatlas, int32_t accumulate) {
    // grid (Gaussian chunks, frames): the frame and its cameras are uniform over the
    // work-group, so the cameras are read with scalar loads
    const int32_t f = (int32_t)blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t v0 = frame_views[f], v1 = frame_views[f + 1];
    const float* P = params + (int64_t)f * C * N + i;
    float rec[11];
#pragma unroll
    for (int k = 0; k < 11; k++) rec[k] = P[(int64_t)k * N];
    double acc[11];
#pragma unroll
    for (int k = 0; k < 11; k++) acc[k] = 0.0;
    // dL/dSigma (world) and dL/do summed over the views: the scale, rotation and
    // activation chains after them are linear and view-independent, so they run
    // once per Gaussian on the sums instead of once per record
    // (dL/dSigma is symmetric: its upper triangle 00, 01, 02, 11, 12, 22 is summed)
    double GSw_sum[6], go_sum = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) GSw_sum[k] = 0.0;
    World w;     // in the view loop only its mean, Sigma and opacity are used
    bool have_world = false;
    // the record's slot sums (0 for culled records): the compositing moments
    // sum dq' (dx, dy, dx^2, dx dy, dy^2) and sum dq', with dq' = alpha dL/dalpha;
    // the next view's are loaded while this view's are used
    float nxt[6];
    auto load6 = [&](int32_t vi) __attribute__((always_inline)) {
        const int64_t gv = (int64_t)view_order[vi] * N + i;
#pragma unroll
        for (int k = 0; k < 6; k++) nxt[k] = grad2d[(int64_t)k * n_gv + gv];
    };
    if (v0 < v1) load6(v0);
    for (int32_t vi = v0; vi < v1; vi++) {
        const int32_t v = view_order[vi];
        const int64_t gv = (int64_t)v * N + i;
        double g6[6];
        bool nz = false;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            g6[k] = (double)nxt[k];
            nz |= (nxt[k] != 0.0f);
        }
        if (vi + 1 < v1) load6(vi + 1);
        if (!nz) continue;
        if (!have_world) {
            world_chain(rec, w);
            have_world = true;
        }
        const ViewDev& V = views[v];
        Cam c;
        if (!camera_chain(V, w, c)) continue;   // never for a record with a gradient: the forward kept it
        // (gradients only from here on: reciprocals instead of divisions)
        const double idet = 1.0 / c.det;
        const double Q00 = c.cp * idet, Q01 = -c.bp * idet, Q11 = c.ap * idet;
        // 2D gradients from the moments (dL/dq = -dq'/2): dL/dm = Q (m0, m1),
        // dL/d(a, b, c) = -(m2 / 2, m3, m4 / 2), and dL/do = sum e dL/dalpha =
        // sum dq' / o (alpha = o e^{-q/2} wherever dq' is not zero); written back
        // as the record's grad2d
        {
            const double m0 = g6[0], m1 = g6[1];
            g6[0] = Q00 * m0 + Q01 * m1;
            g6[1] = Q01 * m0 + Q11 * m1;
            g6[2] = -0.5 * g6[2];
            g6[3] = -g6[3];
            g6[4] = -0.5 * g6[4];
            g6[5] = g6[5] / w.o;
#pragma unroll
            for (int k = 0; k < 6; k++) grad2d[(int64_t)k * n_gv + gv] = (float)g6[k];
        }
        const double G00 = g6[2], G01 = 0.5 * g6[3], G11 = g6[4];
        // QG = Q Gh ; GS = -(QG Q)
        const double QG00 = Q00 * G00 + Q01 * G01, QG01 = Q00 * G01 + Q01 * G11;
        const double QG10 = Q01 * G00 + Q11 * G01, QG11 = Q01 * G01 + Q11 * G11;
        const double GS00 = -(QG00 * Q00 + QG01 * Q01);
        const double GS01 = -(QG00 * Q01 + QG01 * Q11);
        const double GS11 = -(QG10 * Q01 + QG11 * Q11);
        // GJ = GS J (2x3)
        double GJ[6];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            GJ[k] = GS00 * c.J[k] + GS01 * c.J[3 + k];
            GJ[3 + k] = GS01 * c.J[k] + GS11 * c.J[3 + k];
        }
        // dL/dSigma_c = J^T GJ
        double GSc[9];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) GSc[3 * r + k] = c.J[r] * GJ[k] + c.J[3 + r] * GJ[3 + k];
        // dL/dJ = 2 GJ Sigma_c
        double GJm[6];
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int k = 0; k < 3; k++)
                GJm[3 * r + k] = 2.0 * (GJ[3 * r] * c.Sc[k] + GJ[3 * r + 1] * c.Sc[3 + k] + GJ[3 * r + 2] * c.Sc[6 + k]);
        // dL/dSigma = R^T GSc R
        const double* R = V.R;
        double tmp[9], GSw[9];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) tmp[3 * r + k] = GSc[3 * r] * R[k] + GSc[3 * r + 1] * R[3 + k] + GSc[3 * r + 2] * R[6 + k];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int k = r; k < 3; k++) GSw[3 * r + k] = R[r] * tmp[k] + R[3 + r] * tmp[3 + k] + R[6 + r] * tmp[6 + k];
        GSw_sum[0] += GSw[0];
        GSw_sum[1] += GSw[1];
        GSw_sum[2] += GSw[2];
        GSw_sum[3] += GSw[4];
        GSw_sum[4] += GSw[5];
        GSw_sum[5] += GSw[8];
        // mean: dm/dmu_c = J, plus the dependence of J on mu_c
        const double iz = 1.0 / c.zc, iz2 = iz * iz, iz3 = iz2 * iz;
        double gmc0 = c.J[0] * g6[0] + c.J[3] * g6[1];
        double gmc1 = c.J[1] * g6[0] + c.J[4] * g6[1];
        double gmc2 = c.J[2] * g6[0] + c.J[5] * g6[1];
        gmc0 += GJm[2] * (-V.fx * iz2);
        gmc1 += GJm[5] * (-V.fy * iz2);
        gmc2 += GJm[0] * (-V.fx * iz2) + GJm[2] * (2.0 * V.fx * c.xc * iz3) + GJm[4] * (-V.fy * iz2)
                + GJm[5] * (2.0 * V.fy * c.yc * iz3);
#pragma unroll
        for (int k = 0; k < 3; k++) acc[k] += R[k] * gmc0 + R[3 + k] * gmc1 + R[6 + k] * gmc2;
        go_sum += g6[5];
    }
    if (have_world) {
        // The world chain again, so that its rotation, scale and M need no registers
        // during the view loop (the opaque step keeps the compiler from reusing w).
#pragma unroll
        for (int k = 0; k < 11; k++) asm volatile("" : "+v"(rec[k]));
        world_chain(rec, w);
        const double Gs[9] = {GSw_sum[0], GSw_sum[1], GSw_sum[2], GSw_sum[1], GSw_sum[3], GSw_sum[4],
                              GSw_sum[2], GSw_sum[4], GSw_sum[5]};
        // dL/dM = 2 GSw M ; dL/ds (log-scale) ; dL/dRq -> the normalised quaternion -> the stored one
        double gs[3] = {0.0, 0.0, 0.0}, GR[9];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double gm = 2.0 * (Gs[3 * r] * w.M[k] + Gs[3 * r + 1] * w.M[3 + k] +
                                         Gs[3 * r + 2] * w.M[6 + k]);
                gs[k] += gm * w.Rq[3 * r + k];
                GR[3 * r + k] = gm * w.s[k];
            }
        const double qa = w.qh[0], qx = w.qh[1], qy = w.qh[2], qz = w.qh[3];
        double gq[4];
        gq[0] = 2.0 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
        gq[1] = 2.0 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.0 * qx * GR[4] - qa * GR[5] + qz * GR[6] + qa * GR[7]
                       - 2.0 * qx * GR[8]);
        gq[2] = 2.0 * (-2.0 * qy * GR[0] + qx * GR[1] + qa * GR[2] + qx * GR[3] + qz * GR[5] - qa * GR[6] + qz * GR[7]
                       - 2.0 * qy * GR[8]);
        gq[3] = 2.0 * (-2.0 * qz * GR[0] - qa * GR[1] + qx * GR[2] + qa * GR[3] - 2.0 * qz * GR[4] + qy * GR[5]
                       + qx * GR[6] + qy * GR[7]);
        const double qd = gq[0] * qa + gq[1] * qx + gq[2] * qy + gq[3] * qz;
#pragma unroll
        for (int k = 0; k < 3; k++) acc[3 + k] += w.s[k] * gs[k];
#pragma unroll
        for (int k = 0; k < 4; k++) acc[6 + k] += (gq[k] - w.qh[k] * qd) / w.qn;
        acc[10] += go_sum * w.o * (1.0 - w.o);
    }
    const int64_t texel = gauss_texel[i];
    const float m = dyn ? (dyn[texel] ? 1.f : 0.f) : 1.f;
    float* out = gatlas + (int64_t)f * C * HW + texel;
#pragma unroll
    for (int k = 0; k < 11; k++) {
        if (accumulate) out[(int64_t)k * HW] += m * (float)acc[k];
        else out[(int64_t)k * HW] = m * (float)acc[k];
    }
}

// Colour part of the adjoint, FP32: SH coefficient gradients Y_j gc and the
// view-direction term of the position gradient, added to what the geometric
// kernel wrote.  The clamp decision (colour = max(0, 0.5 + sum Y k)) is the
// forward's: the FP32 sum settles it away from 0, and near 0 the forward's
// stored colour (0 exactly where its FP64 sum clamped) is read back.
template <int L>
__global__ __launch_bounds__(128) void k_project_bwd_sh(const ViewDev* __restrict__ views,
                                                        const int32_t* __restrict__ frame_views,
                                                        const int32_t* __restrict__ view_order, int32_t F,
                                                        int32_t C, int64_t N, int64_t n_gv,
                                                        const float* __restrict__ params,
                                                        const pg_splat* __restrict__ splats,
                                                        const float* __restrict__ grad2d,
                                                        const int32_t* __restrict__ gauss_texel,
                                                        const uint8_t* __restrict__ dyn, int64_t HW,
                                                        float* __restrict__ gatlas, int32_t accumulate) {
    constexpr int NB = (L + 1) * (L + 1);
    // grid (Gaussian chunks, frames): the frame and its cameras are uniform over the
    // work-group, so the cameras are read with scalar loads
    const int32_t f = (int32_t)blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t v0 = frame_views[f], v1 = frame_views[f + 1];
    const float* P = params + (int64_t)f * C * N + i;
    World wpos;                      // only mu is used (view direction)
    wpos.mu[0] = P[0];
    wpos.mu[1] = P[N];
    wpos.mu[2] = P[2 * N];
    float sh[3 * NB];
#pragma unroll
    for (int k = 0; k < 3 * NB; k++) sh[k] = P[(int64_t)(11 + k) * N];
    float acc[3 * NB], gmu[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 3 * NB; k++) acc[k] = 0.0f;
    float nxt[3];     // the next view's colour gradients, loaded while this view's are used
    auto load3 = [&](int32_t vi) __attribute__((always_inline)) {
        const int64_t gv = (int64_t)view_order[vi] * N + i;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) nxt[ch] = grad2d[(int64_t)(6 + ch) * n_gv + gv];
    };
    if (v0 < v1) load3(v0);
    for (int32_t vi = v0; vi < v1; vi++) {
        const int32_t v = view_order[vi];
        const float gcol[3] = {nxt[0], nxt[1], nxt[2]};
        if (vi + 1 < v1) load3(vi + 1);
        if (gcol[0] == 0.0f && gcol[1] == 0.0f && gcol[2] == 0.0f) continue;
        const ViewDev& V = views[v];
        double dd64[3], dn64;
        view_dir<L>(V, wpos, dd64, &dn64);
        const float d[3] = {(float)dd64[0], (float)dd64[1], (float)dd64[2]};
        const float dn = (float)dn64;
        float Y[NB];
        sh_basis_f<L>(d[0], d[1], d[2], Y);
        // clamp decision: the FP32 colour sum settles it unless it lies within 1e-3 of the clamp;
        // there the forward's own decision is read back from its colour (max(0, its FP64 sum),
        // stored as float: 0 exactly when it clamped), instead of forming the FP64 sum again
        // (whose sixteen doubles doubled this kernel's registers)
        float gc[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float raw = 0.5f;
#pragma unroll
            for (int j = 0; j < NB; j++) raw = fmaf(Y[j], sh[3 * j + ch], raw);
            bool clamped = raw < 0.0f;
            if (fabsf(raw) < 1e-3f) clamped = !(splats[(int64_t)v * N + i].color[ch] > 0.0f);
            gc[ch] = clamped ? 0.0f : gcol[ch];   // clamped channel: no gradient
        }
        // SH coefficients: dL/dk[j][ch] = Y_j gc_ch; direction: sum_j (sum_ch k[j][ch] gc_ch) grad Y_j
        float wj[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) {
#pragma unroll
            for (int ch = 0; ch < 3; ch++) acc[3 * j + ch] += Y[j] * gc[ch];
            wj[j] = (sh[3 * j] * gc[0] + sh[3 * j + 1] * gc[1]) + sh[3 * j + 2] * gc[2];
        }
        float gd[3];
        sh_grad_dot_f<L>(d[0], d[1], d[2], wj, gd);
        const float dd = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
#pragma unroll
        for (int k = 0; k < 3; k++) gmu[k] += (gd[k] - d[k] * dd) / dn;
    }
    const int64_t texel = gauss_texel[i];
    const float m = dyn ? (dyn[texel] ? 1.f : 0.f) : 1.f;
    float* out = gatlas + (int64_t)f * C * HW + texel;
#pragma unroll
    for (int k = 0; k < 3; k++) out[(int64_t)k * HW] += m * gmu[k];   // after the geometric kernel
#pragma unroll
    for (int k = 0; k < 3 * NB; k++) {
        if (accumulate) out[(int64_t)(11 + k) * HW] += m * acc[k];
        else out[(int64_t)(11 + k) * HW] = m * acc[k];
    }
}

// Per-record sums of the instance slots.  Slots are laid out record by
// record in (view, id) order, so one work-group takes 256 consecutive
// records, whose slots form one contiguous range; the group streams it
// through LDS in coalesced chunks (ten independent loads per thread in
// flight) while each thread adds its own record's slots in rectangle
// row-major order, and grad2d is written coalesced.  A slot counts only when
// its tag is this sort's generation (the adjoint wrote it in this step);
// after an overflowed sort there are no slots and every sum is 0.
constexpr int kSumRecs = 256;
constexpr int kSumChunk = 256;    // instances per LDS chunk (10 KiB)

__global__ __launch_bounds__(kSumRecs) void k_slot_sum(const pg_bin* __restrict__ bins,
                                                       const int32_t* __restrict__ inst_first,
                                                       const int64_t* __restrict__ n_inst_dev, int64_t cap,
                                                       const float* __restrict__ inst_grad, int64_t n_gv,
                                                       float* __restrict__ grad2d) {
    __shared__ float s_g[kSumChunk * kSlotWords];
    __shared__ int64_t s_range[2];
    const int64_t g0 = (int64_t)blockIdx.x * kSumRecs;
    const int64_t gv = g0 + threadIdx.x;
    const int64_t glast = imin(g0 + kSumRecs, n_gv) - 1;
    const bool sorted_ok = *n_inst_dev <= cap;
    const uint32_t gen = (uint32_t)n_inst_dev[1];
    int32_t nt = 0;
    int64_t first = 0;
    if (gv <= glast && sorted_ok) {
        // the record's kept tiles from the slot offsets (an exclusive scan of them over
        // every record), so the 16-byte bins need not be read
        first = inst_first[gv];
        const int64_t next = gv + 1 < n_gv ? (int64_t)inst_first[gv + 1] : *n_inst_dev;
        nt = (int32_t)(next - first);
    }
    if (gv == g0) s_range[0] = first;
    if (gv == glast) s_range[1] = first + nt;
    __syncthreads();
    const int64_t e0 = s_range[0], e1 = s_range[1];
    float s9[9];
#pragma unroll
    for (int k = 0; k < 9; k++) s9[k] = 0.0f;
    for (int64_t c0 = e0; c0 < e1; c0 += kSumChunk) {
        const int64_t c1 = imin(e1, c0 + kSumChunk);
        const int32_t nw = (int32_t)((c1 - c0) * kSlotWords);
        __syncthreads();
        const float* src = inst_grad + c0 * kSlotWords;
        float x[kSlotWords];
#pragma unroll
        for (int r = 0; r < kSlotWords; r++) {
            const int32_t w = r * kSumRecs + threadIdx.x;
            x[r] = w < nw ? src[w] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < kSlotWords; r++) s_g[r * kSumRecs + threadIdx.x] = x[r];
        __syncthreads();
        const int32_t a = (int32_t)(imax(first, c0) - c0), b = (int32_t)(imin(first + nt, c1) - c0);
        for (int32_t u = a; u < b; u++) {
            if (__float_as_uint(s_g[u * kSlotWords + kSlotWords - 1]) != gen) continue;   // not written this step
#pragma unroll
            for (int k = 0; k < 9; k++) s9[k] += s_g[u * kSlotWords + k];
        }
    }
    if (gv <= glast) {
#pragma unroll
        for (int k = 0; k < 9; k++) grad2d[(int64_t)k * n_gv + gv] = s9[k];
    }
}

}  // namespace

hipError_t launch_flow_mask(const pg_views* v, const float* params, const uint8_t* masks, uint8_t* tile_motion,
                            uint8_t* dyn_gauss, const int32_t* texel_gauss, int64_t HW, uint8_t* dyn_texel,
                            uint64_t* counters, hipStream_t s) {
    const int64_t nfn = (int64_t)v->frames * v->n_gauss;
    if (nfn > 0) k_fill_u8<<<(unsigned)ceil_div(nfn, 256), 256, 0, s>>>(dyn_gauss, nfn);
    if (v->n_tiles > 0)
        k_tile_motion<<<(unsigned)v->n_tiles, 64, 0, s>>>(v->d_views, v->n_views, v->n_tiles, v->tiling.tile_w,
                                                          v->tiling.tile_h, masks, tile_motion);
    if (v->n_gv > 0)
        k_flow_mask<<<(unsigned)(v->n_views * ceil_div(v->n_gauss, 128)), 128, 0, s>>>(
            v->d_views, v->channels, v->n_gauss, v->n_gv, v->tiling.tile_w, v->tiling.tile_h, params, masks,
            tile_motion, dyn_gauss, reinterpret_cast<unsigned long long*>(counters));
    if (dyn_texel && HW > 0)
        k_dyn_texel<<<(unsigned)ceil_div(HW, 256), 256, 0, s>>>(dyn_gauss, texel_gauss, HW, v->frames, v->n_gauss,
                                                               dyn_texel);
    return hipGetLastError();
}

hipError_t launch_project(const pg_views* v, const float* params, pg_splat* splats, pg_bin* bins,
                          pg_tile_set* tiles, uint8_t* visible, hipStream_t s) {
    const int64_t n = (int64_t)v->frames * v->n_gauss;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)ceil_div(v->n_gauss, 128), (unsigned)v->frames);
    auto args = [&](auto kern) {
        kern<<<grid, 128, 0, s>>>(v->d_views, v->d_frame_views, v->d_view_order, v->frames, v->channels, v->n_gauss,
                                  v->tiling.tile_w, v->tiling.tile_h, params, splats, bins, tiles, visible);
    };
    switch (v->sh_degree) {
        case 0: args(k_project<0>); break;
        case 1: args(k_project<1>); break;
        case 2: args(k_project<2>); break;
        default: args(k_project<3>); break;
    }
    return hipGetLastError();
}

hipError_t launch_slot_sum(const pg_views* v, const pg_bin* bins, const int32_t* inst_first,
                           const int64_t* n_inst_dev, int64_t cap, const float* inst_grad, float* grad2d,
                           hipStream_t s) {
    if (v->n_gv == 0) return hipSuccess;
    const unsigned grid = (unsigned)ceil_div(v->n_gv, kSumRecs);
    k_slot_sum<<<grid, kSumRecs, 0, s>>>(bins, inst_first, n_inst_dev, cap, inst_grad, v->n_gv, grad2d);
    return hipGetLastError();
}

hipError_t launch_project_bwd(const pg_views* v, const float* params, const pg_splat* splats, float* grad2d,
                              const int32_t* gauss_texel, const uint8_t* dyn, int32_t H, int32_t W,
                              float* dL_datlas, int32_t accumulate, hipStream_t s) {
    const int64_t HW = (int64_t)H * W;
    if (!accumulate) {
        hipError_t e = fill_u32(dL_datlas, 0u, (int64_t)v->frames * v->channels * HW, s);
        if (e != hipSuccess) return e;
    }
    const int64_t n = (int64_t)v->frames * v->n_gauss;
    if (n == 0) return hipGetLastError();
    const dim3 grid((unsigned)ceil_div(v->n_gauss, 128), (unsigned)v->frames);
    k_project_bwd_geo<<<grid, 128, 0, s>>>(v->d_views, v->d_frame_views, v->d_view_order, v->frames, v->channels,
                                           v->n_gauss, v->n_gv, params, grad2d, gauss_texel, dyn, HW, dL_datlas,
                                           accumulate);
    auto args = [&](auto kern) {
        kern<<<grid, 128, 0, s>>>(v->d_views, v->d_frame_views, v->d_view_order, v->frames, v->channels, v->n_gauss,
                                  v->n_gv, params, splats, grad2d, gauss_texel, dyn, HW, dL_datlas, accumulate);
    };
    switch (v->sh_degree) {
        case 0: args(k_project_bwd_sh<0>); break;
        case 1: args(k_project_bwd_sh<1>); break;
        case 2: args(k_project_bwd_sh<2>); break;
        default: args(k_project_bwd_sh<3>); break;
    }
    return hipGetLastError();
}

}  // namespace pg
