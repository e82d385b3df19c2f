// UV-based pruning (Sec. 4.2 "UV-Based Pruning"; UV projection equation of
// Sec. 3).  A Gaussian's position in spherical coordinates gives its UV pixel
//   u = floor((pi + atan2(y, x)) / (2 pi) M),  v = floor(acos(z / rho) / pi N)
// (FP64; theta = pi wraps to u = 0, phi = pi stays in the last row, rho = 0
// is invalid).  Valid UV projection: with the pixel of the storing texel
// given, a Gaussian that maps elsewhere is invalid.  Max-K: per frame and
// pixel, the K valid Gaussians of highest opacity are kept (by the logit,
// which orders like the opacity; ties by ascending id).
//
// A segmented top-K by two stable radix sorts of (key, index) pairs: first by
// the opacity (largest first), then by (frame, pixel), so each pixel's run
// comes out ordered by opacity and then id; a Gaussian's rank is its distance
// from the start of its run.
#include "pg_internal.h"

namespace pg {

namespace {

constexpr int kT = 256;

// float -> uint32 whose ascending order is the float's descending order
// (-0 counts as +0, as in a float comparison)
__device__ __forceinline__ uint32_t desc_key(float x) {
    if (x == 0.0f) x = 0.0f;
    const uint32_t b = __float_as_uint(x);
    const uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ~asc;
}

__global__ void k_uv_count(const int64_t* __restrict__ n_dev, int64_t n_cap, int32_t F, int64_t* __restrict__ cnt) {
    cnt[0] = (int64_t)F * imin(*n_dev, n_cap);
}

__global__ __launch_bounds__(kT) void k_uv_key(const float* __restrict__ params, const int64_t* __restrict__ n_dev,
                                               int64_t n_cap, int32_t F, int32_t C, int32_t M, int32_t Nv,
                                               const int32_t* __restrict__ expected, int32_t* __restrict__ uv,
                                               uint32_t* __restrict__ okey, int32_t* __restrict__ oval) {
    const int64_t n = imin(*n_dev, n_cap);
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= (int64_t)F * n) return;
    const int32_t f = (int32_t)(j / n);
    const int64_t i = j - (int64_t)f * n;
    const float* P = params + (int64_t)f * C * n_cap + i;
    const double x = P[0], y = P[n_cap], z = P[2 * n_cap];
    const double rho = sqrt((x * x + y * y) + z * z);
    int32_t key = -1;
    if (rho > 0.0) {
        const double theta = atan2(y, x);
        double c = z / rho;
        c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
        const double phi = acos(c);
        int64_t u = (int64_t)floor((3.141592653589793 + theta) / (2.0 * 3.141592653589793) * (double)M);
        int64_t v = (int64_t)floor(phi / 3.141592653589793 * (double)Nv);
        if (u >= M) u -= M;
        if (v >= Nv) v = Nv - 1;
        key = (int32_t)(v * M + u);
        if (expected && expected[(int64_t)f * n_cap + i] != key) key = -1;
    }
    const int64_t g = (int64_t)f * n_cap + i;
    uv[g] = key;
    okey[j] = key >= 0 ? desc_key(P[10 * n_cap]) : 0xFFFFFFFFu;
    oval[j] = (int32_t)g;
}

// records in opacity order -> (frame, pixel) keys; invalid ones get F M Nv
__global__ __launch_bounds__(kT) void k_uv_emit(const int32_t* __restrict__ oval, const int64_t* __restrict__ cnt,
                                                int64_t n_cap, int32_t M, int32_t Nv, int32_t F,
                                                const int32_t* __restrict__ uv, uint32_t* __restrict__ pkey,
                                                int32_t* __restrict__ pval) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= cnt[0]) return;
    const int32_t g = oval[j];
    const int32_t f = (int32_t)(g / n_cap);
    const int32_t u = uv[g];
    pkey[j] = u >= 0 ? (uint32_t)((int64_t)f * M * Nv + u) : (uint32_t)((int64_t)F * M * Nv);
    pval[j] = g;
}

__global__ __launch_bounds__(kT) void k_uv_start(const uint32_t* __restrict__ pkey, const int64_t* __restrict__ cnt,
                                                 int32_t* __restrict__ start) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= cnt[0]) return;
    if (j == 0 || pkey[j] != pkey[j - 1]) start[pkey[j]] = (int32_t)j;
}

__global__ __launch_bounds__(kT) void k_uv_rank(const uint32_t* __restrict__ pkey, const int32_t* __restrict__ pval,
                                                const int64_t* __restrict__ cnt, const int32_t* __restrict__ start,
                                                uint32_t sentinel, int32_t K, int32_t* __restrict__ rank,
                                                uint8_t* __restrict__ keep) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= cnt[0]) return;
    const uint32_t key = pkey[j];
    const int32_t g = pval[j];
    if (key == sentinel) {
        rank[g] = -1;
        keep[g] = 0;
        return;
    }
    const int32_t r = (int32_t)j - start[key];
    rank[g] = r;
    keep[g] = r < K ? 1 : 0;
}

int key_bits_for(int64_t n_keys) {
    int b = 1;
    while (((int64_t)1 << b) < n_keys) b++;
    return b;
}

struct UvWs {
    int64_t* cnt;
    uint32_t *ka, *kb;
    int32_t *va, *vb, *start;
    void* sort_ws;
};

UvWs carve_uv(int64_t n_cap, int32_t F, int32_t M, int32_t Nv, void* ws, size_t* total) {
    const int64_t n = imax((int64_t)F * n_cap, 1);
    char* p = (char*)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = p + off;
        off += align256(bytes);
        return q;
    };
    UvWs w{};
    w.cnt = (int64_t*)take(8);
    w.ka = (uint32_t*)take(n * 4);
    w.kb = (uint32_t*)take(n * 4);
    w.va = (int32_t*)take(n * 4);
    w.vb = (int32_t*)take(n * 4);
    w.start = (int32_t*)take(((int64_t)F * M * Nv + 1) * 4);
    const int bits = imax(32, key_bits_for((int64_t)F * M * Nv + 1));
    w.sort_ws = take(sort_pairs_ws_bytes(n, bits));
    if (total) *total = off;
    return w;
}

}  // namespace

size_t uv_prune_ws_bytes(int64_t n_cap, int32_t F, int32_t M, int32_t Nv) {
    size_t total = 0;
    carve_uv(n_cap, F, M, Nv, nullptr, &total);
    return total;
}

hipError_t launch_uv_prune(const float* params, const int64_t* n_dev, int64_t n_cap, int32_t F, int32_t C, int32_t M,
                           int32_t Nv, int32_t K, const int32_t* expected, int32_t* uv, int32_t* rank, uint8_t* keep,
                           void* ws, hipStream_t s) {
    UvWs w = carve_uv(n_cap, F, M, Nv, ws, nullptr);
    const int64_t n = (int64_t)F * n_cap;
    k_uv_count<<<1, 1, 0, s>>>(n_dev, n_cap, F, w.cnt);
    if (n == 0) return hipGetLastError();
    const unsigned grid = (unsigned)ceil_div(n, kT);
    k_uv_key<<<grid, kT, 0, s>>>(params, n_dev, n_cap, F, C, M, Nv, expected, uv, w.ka, w.va);
    uint32_t* ok;
    int32_t* ov;
    hipError_t e = sort_pairs(w.ka, w.va, w.kb, w.vb, w.cnt, n, 32, w.sort_ws, &ok, &ov, s);
    if (e != hipSuccess) return e;
    // the pixel keys go to the pair the opacity order does not occupy
    uint32_t* pk = ok == w.ka ? w.kb : w.ka;
    int32_t* pv = ov == w.va ? w.vb : w.va;
    k_uv_emit<<<grid, kT, 0, s>>>(ov, w.cnt, n_cap, M, Nv, F, uv, pk, pv);
    const uint32_t sentinel = (uint32_t)((int64_t)F * M * Nv);
    uint32_t* sk;
    int32_t* sv;
    e = sort_pairs(pk, pv, ok, ov, w.cnt, n, key_bits_for((int64_t)sentinel + 1), w.sort_ws, &sk, &sv, s);
    if (e != hipSuccess) return e;
    k_uv_start<<<grid, kT, 0, s>>>(sk, w.cnt, w.start);
    k_uv_rank<<<grid, kT, 0, s>>>(sk, sv, w.cnt, w.start, sentinel, K, rank, keep);
    return hipGetLastError();
}

}  // namespace pg
