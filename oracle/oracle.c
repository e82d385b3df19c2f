/*
 * oracle.c -- plain FP64 CPU oracle for the PackUV-GS differentiable
 * splatting path (atlas fetch, EWA projection, tile binning with depth
 * sort, front-to-back compositing, and its adjoint back to the atlas).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a slow, obviously-correct
 * restatement of the method used to check the GPU library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source with the GPU library: the two agree only because they
 * implement the same formulas.
 *
 * Sources (PackUV, arXiv 2602.23040):
 *   - Gaussian record (mu, covariance from scale and rotation, opacity, SH
 *     colour): Sec. 3 "Preliminaries", 3DGS paragraph.
 *   - Texel storage of the record: Sec. 4.2 "Fitting UV Maps Directly".
 *   - EWA projection Sigma2D = J W Sigma W^T J^T, the Jacobian, the +0.3
 *     low-pass, det/z validity test, lambda_max and the 3-sigma radius:
 *     "Covariance-Aware Gaussian Masking" (Sec. 4.2) and Algorithm 1
 *     (steps 1-4); viewer projection X_c = R X + t (supplementary, viewer).
 *   - Per-pixel footprint d^2 <= 9: Sec. 4.2 masking equation / Alg. 1 step 5.
 *   - Compositing C = sum_i T_i alpha_i c_i, T_i = prod_{j<i} (1 - alpha_j):
 *     supplementary, viewer section (the formula is front to back).
 *   - Gradient freezing grad <- D_i grad: Sec. 4.2 "Gradient Freezing".
 *   - Photometric objective (1 - lambda_ssim) L1 + lambda_ssim (1 - SSIM),
 *     scale and opacity regularisers: Sec. 4.2 "Objective".
 *   - Sparse Adam on FP32 master weights: Sec. 4.3 LPO paragraph.
 *   - UV-based pruning (valid UV projection, top-K by opacity per UV pixel):
 *     Sec. 4.2 pruning paragraph and the UV projection equation of Sec. 3.
 *   - Covariance-aware flow masking (dynamic label per Gaussian, OR across
 *     cameras): Sec. 4.2 masking paragraph and Algorithm 1.
 *   - LPO fake quantiser (uniform K-bit proxy, straight-through gradient,
 *     per-channel min/max scale): Sec. 4.3 LPO paragraph, supplementary
 *     low-precision training and video-coding sections.
 * Where the paper is silent (alpha rule, termination, SH basis, camera axes,
 * activations, tie-breaks) the readings listed in the design notes are used;
 * each is restated next to the code that takes it.
 *
 * Everything is FP64.  Decision quantities (camera-space mean, covariances,
 * det, lambda_max, radius, pixel mean, tile rectangle, depth key) follow a
 * fixed evaluation order with no contraction (build with
 * -ffp-contract=off -fno-fast-math), so that an independent implementation
 * using the same order reaches the same bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ types */

typedef struct {
    double R[9];          /* world -> camera rotation, row-major; x_c = R x + t */
    double t[3];
    double fx, fy, cx, cy;
    int32_t width, height, frame, reserved;
} or_camera;

typedef struct {
    int32_t valid;        /* survived the z / det culls and its tile rectangle is not empty */
    int32_t radius;       /* ceil(3 sqrt(lambda_max)) */
    int32_t rect[4];      /* x_lo, y_lo, x_hi, y_hi inclusive tile indices */
    uint32_t key;         /* bit pattern of fp32(z_c) */
    uint32_t pad;
    double z;             /* camera-space depth z_c */
    double mean[2];       /* pixel-space mean */
    double cov2d[3];      /* a', b', c' of Sigma2D incl. low-pass */
    double det;
    double conic[3];      /* inverse of Sigma2D: (a, b, c) with q = a dx^2 + 2 b dx dy + c dy^2 */
    double opacity;
    double color[3];      /* max(0, raw) */
    double color_raw[3];  /* 0.5 + sum_j Y_j k_j */
    int32_t visible;      /* survived the z / det culls and the square of half-side r around the mean
                             reaches a pixel of the image (the rectangle with one-pixel tiles) */
    int32_t pad2;
    int64_t n_tiles;      /* tiles of the rectangle: the Gaussian is listed in every one */
} or_proj;

typedef struct {
    int64_t tile;
    uint32_t key;
    int32_t id;
} or_inst;

#define OR_NEAR_Z 0.2
#define OR_LOWPASS 0.3
#define OR_DET_MIN 1e-7
#define OR_Q_MAX 9.0
#define OR_ALPHA_MAX 0.99
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_T_MIN 1e-4

/* ------------------------------------------------------------------ SH basis
 * Real spherical harmonics up to degree 3 with the Condon-Shortley phase
 * kept, as functions of a unit direction d = (x, y, z).  Constants are the
 * normalisations sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) of each (l, m), times the
 * sqrt(2) of the real combination, written as closed forms. */

static double SHC[16];

static void sh_init(void) {
    static int done = 0;
    if (done) return;
    const double pi = 3.14159265358979323846;
    SHC[0] = 0.5 * sqrt(1.0 / pi);
    SHC[1] = sqrt(3.0 / (4.0 * pi));
    SHC[2] = 0.5 * sqrt(15.0 / pi);          /* xy, yz, xz */
    SHC[3] = 0.25 * sqrt(5.0 / pi);          /* 3z^2 - 1 */
    SHC[4] = 0.25 * sqrt(15.0 / pi);         /* x^2 - y^2 */
    SHC[5] = 0.25 * sqrt(35.0 / (2.0 * pi)); /* y(3x^2 - y^2), x(x^2 - 3y^2) */
    SHC[6] = 0.5 * sqrt(105.0 / pi);         /* xyz */
    SHC[7] = 0.25 * sqrt(21.0 / (2.0 * pi)); /* y(5z^2 - 1), x(5z^2 - 1) */
    SHC[8] = 0.25 * sqrt(7.0 / pi);          /* z(5z^2 - 3) */
    SHC[9] = 0.25 * sqrt(105.0 / pi);        /* z(x^2 - y^2) */
    done = 1;
}

/* Y[j], j = l^2 + l + m, and optionally dY[j][3] = gradient of the polynomial. */
static void sh_eval(const double d[3], int L, double* Y, double (*dY)[3]) {
    const double x = d[0], y = d[1], z = d[2];
    int nb = (L + 1) * (L + 1);
    for (int j = 0; j < nb; j++) {
        Y[j] = 0.0;
        if (dY) dY[j][0] = dY[j][1] = dY[j][2] = 0.0;
    }
    Y[0] = SHC[0];
    if (L >= 1) {
        Y[1] = -SHC[1] * y;
        Y[2] = SHC[1] * z;
        Y[3] = -SHC[1] * x;
        if (dY) {
            dY[1][1] = -SHC[1];
            dY[2][2] = SHC[1];
            dY[3][0] = -SHC[1];
        }
    }
    if (L >= 2) {
        Y[4] = SHC[2] * x * y;
        Y[5] = -SHC[2] * y * z;
        Y[6] = SHC[3] * (3.0 * z * z - 1.0);
        Y[7] = -SHC[2] * x * z;
        Y[8] = SHC[4] * (x * x - y * y);
        if (dY) {
            dY[4][0] = SHC[2] * y;  dY[4][1] = SHC[2] * x;
            dY[5][1] = -SHC[2] * z; dY[5][2] = -SHC[2] * y;
            dY[6][2] = 6.0 * SHC[3] * z;
            dY[7][0] = -SHC[2] * z; dY[7][2] = -SHC[2] * x;
            dY[8][0] = 2.0 * SHC[4] * x; dY[8][1] = -2.0 * SHC[4] * y;
        }
    }
    if (L >= 3) {
        Y[9] = -SHC[5] * y * (3.0 * x * x - y * y);
        Y[10] = SHC[6] * x * y * z;
        Y[11] = -SHC[7] * y * (5.0 * z * z - 1.0);
        Y[12] = SHC[8] * z * (5.0 * z * z - 3.0);
        Y[13] = -SHC[7] * x * (5.0 * z * z - 1.0);
        Y[14] = SHC[9] * z * (x * x - y * y);
        Y[15] = -SHC[5] * x * (x * x - 3.0 * y * y);
        if (dY) {
            dY[9][0] = -6.0 * SHC[5] * x * y;
            dY[9][1] = -SHC[5] * (3.0 * x * x - 3.0 * y * y);
            dY[10][0] = SHC[6] * y * z; dY[10][1] = SHC[6] * x * z; dY[10][2] = SHC[6] * x * y;
            dY[11][1] = -SHC[7] * (5.0 * z * z - 1.0); dY[11][2] = -10.0 * SHC[7] * y * z;
            dY[12][2] = SHC[8] * (15.0 * z * z - 3.0);
            dY[13][0] = -SHC[7] * (5.0 * z * z - 1.0); dY[13][2] = -10.0 * SHC[7] * x * z;
            dY[14][0] = 2.0 * SHC[9] * x * z; dY[14][1] = -2.0 * SHC[9] * y * z;
            dY[14][2] = SHC[9] * (x * x - y * y);
            dY[15][0] = -SHC[5] * (3.0 * x * x - 3.0 * y * y); dY[15][1] = 6.0 * SHC[5] * x * y;
        }
    }
}

void or_sh_basis(const double* dirs, int64_t n, int32_t L, double* out) {
    sh_init();
    int nb = (L + 1) * (L + 1);
    for (int64_t i = 0; i < n; i++) sh_eval(dirs + 3 * i, L, out + nb * i, NULL);
}

/* ------------------------------------------------------------------ fetch
 * Occupied texels, in row-major (y, then x) order, are the Gaussians of a
 * frame; their id is their rank.  The record's channels are copied to FP64
 * planes P[f][c][i]. */

int64_t or_fetch(const float* atlas, const uint8_t* occ, int32_t F, int32_t C, int32_t H, int32_t W,
                 int32_t* ids, double* params) {
    int64_t HW = (int64_t)H * W, n = 0;
    for (int64_t p = 0; p < HW; p++)
        if (occ[p]) ids[n++] = (int32_t)p;
    for (int32_t f = 0; f < F; f++)
        for (int32_t c = 0; c < C; c++) {
            const float* plane = atlas + ((int64_t)f * C + c) * HW;
            double* dst = params + ((int64_t)f * C + c) * n;
            for (int64_t i = 0; i < n; i++) dst[i] = (double)plane[ids[i]];
        }
    return n;
}

/* ------------------------------------------------------------------ projection */

typedef struct {
    double mu[3], s[3], qn, qh[4], o;
    double Rq[9], M[9], S[9];
    double xc, yc, zc;
    double A[9], Sc[9], J[6], T[6];
    double ap, bp, cp, det;
} or_chain;

static void quat_to_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Activations (s = exp(l_s), unit quaternion, o = sigmoid(l_o)) and the
 * world covariance Sigma = R(q) diag(s)^2 R(q)^T = M M^T with M = R(q) diag(s). */
static void chain_world(const double* P, int64_t N, int64_t i, or_chain* c) {
    for (int k = 0; k < 3; k++) c->mu[k] = P[k * N + i];
    for (int k = 0; k < 3; k++) c->s[k] = exp(P[(3 + k) * N + i]);
    double qw = P[6 * N + i], qx = P[7 * N + i], qy = P[8 * N + i], qz = P[9 * N + i];
    c->qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    c->qh[0] = qw / c->qn; c->qh[1] = qx / c->qn; c->qh[2] = qy / c->qn; c->qh[3] = qz / c->qn;
    c->o = 1.0 / (1.0 + exp(-P[10 * N + i]));
    quat_to_rot(c->qh, c->Rq);
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) c->M[3 * r + k] = c->Rq[3 * r + k] * c->s[k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            c->S[3 * r + k] = (c->M[3 * r] * c->M[3 * k] + c->M[3 * r + 1] * c->M[3 * k + 1])
                              + c->M[3 * r + 2] * c->M[3 * k + 2];
}

/* Camera part of the chain: mu_c = R mu + t; Sigma_c = R Sigma R^T;
 * J at mu_c; Sigma2D = J Sigma_c J^T + 0.3 I.  Returns 0 when culled by z. */
static int chain_camera(const or_camera* cam, or_chain* c) {
    const double* R = cam->R;
    c->xc = ((R[0] * c->mu[0] + R[1] * c->mu[1]) + R[2] * c->mu[2]) + cam->t[0];
    c->yc = ((R[3] * c->mu[0] + R[4] * c->mu[1]) + R[5] * c->mu[2]) + cam->t[1];
    c->zc = ((R[6] * c->mu[0] + R[7] * c->mu[1]) + R[8] * c->mu[2]) + cam->t[2];
    if (!(c->zc > OR_NEAR_Z)) return 0;
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            c->A[3 * r + k] = (R[3 * r] * c->S[k] + R[3 * r + 1] * c->S[3 + k]) + R[3 * r + 2] * c->S[6 + k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            c->Sc[3 * r + k] = (c->A[3 * r] * R[3 * k] + c->A[3 * r + 1] * R[3 * k + 1]) + c->A[3 * r + 2] * R[3 * k + 2];
    const double z2 = c->zc * c->zc;
    c->J[0] = cam->fx / c->zc;
    c->J[1] = 0.0;
    c->J[2] = -(cam->fx * c->xc) / z2;
    c->J[3] = 0.0;
    c->J[4] = cam->fy / c->zc;
    c->J[5] = -(cam->fy * c->yc) / z2;
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            c->T[3 * r + k] = (c->J[3 * r] * c->Sc[k] + c->J[3 * r + 1] * c->Sc[3 + k]) + c->J[3 * r + 2] * c->Sc[6 + k];
    double s00 = (c->T[0] * c->J[0] + c->T[1] * c->J[1]) + c->T[2] * c->J[2];
    double s01 = (c->T[0] * c->J[3] + c->T[1] * c->J[4]) + c->T[2] * c->J[5];
    double s11 = (c->T[3] * c->J[3] + c->T[4] * c->J[4]) + c->T[5] * c->J[5];
    c->ap = s00 + OR_LOWPASS;
    c->bp = s01;
    c->cp = s11 + OR_LOWPASS;
    c->det = c->ap * c->cp - c->bp * c->bp;
    return 1;
}

static void camera_centre(const or_camera* cam, double cw[3]) {
    const double* R = cam->R;
    for (int k = 0; k < 3; k++) cw[k] = -((R[k] * cam->t[0] + R[3 + k] * cam->t[1]) + R[6 + k] * cam->t[2]);
}

static void project_one(const double* P, int64_t N, int64_t i, int32_t L, const or_camera* cam,
                        int32_t tw, int32_t th, or_proj* o) {
    memset(o, 0, sizeof *o);
    or_chain c;
    chain_world(P, N, i, &c);
    o->opacity = c.o;
    if (!chain_camera(cam, &c)) { o->z = c.zc; return; }
    o->z = c.zc;
    o->cov2d[0] = c.ap; o->cov2d[1] = c.bp; o->cov2d[2] = c.cp;
    o->det = c.det;
    if (!(c.det > OR_DET_MIN)) return;
    const double tr = c.ap + c.cp;
    const double lam = 0.5 * (tr + sqrt(fmax(0.0, tr * tr - 4.0 * c.det)));
    const double rr = ceil(3.0 * sqrt(lam));
    o->radius = (int32_t)rr;
    o->mean[0] = (cam->fx * c.xc) / c.zc + cam->cx;
    o->mean[1] = (cam->fy * c.yc) / c.zc + cam->cy;
    const int32_t TX = (cam->width + tw - 1) / tw, TY = (cam->height + th - 1) / th;
    double xlo = fmax(0.0, floor((o->mean[0] - rr) / tw));
    double xhi = fmin((double)(TX - 1), floor((o->mean[0] + rr) / tw));
    double ylo = fmax(0.0, floor((o->mean[1] - rr) / th));
    double yhi = fmin((double)(TY - 1), floor((o->mean[1] + rr) / th));
    o->conic[0] = c.cp / c.det;
    o->conic[1] = -c.bp / c.det;
    o->conic[2] = c.ap / c.det;
    float zf = (float)c.zc;
    memcpy(&o->key, &zf, 4);
    /* view-dependent colour: d = (mu - c_w)/|mu - c_w|, colour = max(0, 0.5 + sum Y k) */
    double cw[3], d[3], Y[16];
    camera_centre(cam, cw);
    for (int k = 0; k < 3; k++) d[k] = c.mu[k] - cw[k];
    double dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    for (int k = 0; k < 3; k++) d[k] /= dn;
    sh_eval(d, L, Y, NULL);
    int nb = (L + 1) * (L + 1);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int j = 0; j < nb; j++) acc += Y[j] * P[(11 + 3 * j + ch) * N + i];
        o->color_raw[ch] = 0.5 + acc;
        o->color[ch] = o->color_raw[ch] > 0.0 ? o->color_raw[ch] : 0.0;
    }
    /* Visibility, the set sparse Adam updates: the rectangle the same formula
     * gives with one-pixel tiles is not empty, i.e. some pixel of the image lies
     * within r of the mean on both axes.  It does not depend on the tile shape. */
    const double pxlo = fmax(0.0, floor(o->mean[0] - rr)), pxhi = fmin((double)(cam->width - 1), floor(o->mean[0] + rr));
    const double pylo = fmax(0.0, floor(o->mean[1] - rr)), pyhi = fmin((double)(cam->height - 1), floor(o->mean[1] + rr));
    o->visible = pxlo <= pxhi && pylo <= pyhi;
    if (xlo > xhi || ylo > yhi) return;
    o->rect[0] = (int32_t)xlo; o->rect[1] = (int32_t)ylo;
    o->rect[2] = (int32_t)xhi; o->rect[3] = (int32_t)yhi;
    o->n_tiles = (int64_t)(o->rect[2] - o->rect[0] + 1) * (o->rect[3] - o->rect[1] + 1);
    o->valid = 1;
}

void or_project(const double* P, int64_t N, int32_t C, int32_t L, const or_camera* cam,
                int32_t tw, int32_t th, or_proj* out) {
    (void)C;
    sh_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) project_one(P, N, i, L, cam, tw, th, &out[i]);
}

static int64_t n_tiles_of(const or_proj* p) { return p->valid ? p->n_tiles : 0; }

int64_t or_count_instances(const or_proj* pr, int64_t N) {
    int64_t s = 0;
    for (int64_t i = 0; i < N; i++) s += n_tiles_of(&pr[i]);
    return s;
}

/* ------------------------------------------------------------------ bin + sort
 * Each surviving Gaussian is listed in every tile of its rectangle; lists are
 * ordered by (tile, depth key, id) -- front to back by camera-space depth,
 * equal depths by ascending id. */

static int inst_cmp(const void* a, const void* b) {
    const or_inst* x = (const or_inst*)a;
    const or_inst* y = (const or_inst*)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

void or_bin_sort(const or_proj* pr, int64_t N, const or_camera* cam, int32_t tw, int32_t th,
                 or_inst* inst, int64_t* ranges) {
    const int32_t TX = (cam->width + tw - 1) / tw, TY = (cam->height + th - 1) / th;
    int64_t k = 0;
    for (int64_t i = 0; i < N; i++) {
        if (!pr[i].valid) continue;
        for (int32_t ty = pr[i].rect[1]; ty <= pr[i].rect[3]; ty++)
            for (int32_t tx = pr[i].rect[0]; tx <= pr[i].rect[2]; tx++) {
                inst[k].tile = (int64_t)ty * TX + tx;
                inst[k].key = pr[i].key;
                inst[k].id = (int32_t)i;
                k++;
            }
    }
    qsort(inst, (size_t)k, sizeof(or_inst), inst_cmp);
    const int64_t T = (int64_t)TX * TY;
    for (int64_t t = 0; t < 2 * T; t++) ranges[t] = 0;
    for (int64_t j = 0; j < k; j++) {
        int64_t t = inst[j].tile;
        if (j == 0 || inst[j - 1].tile != t) ranges[2 * t] = j;
        if (j == k - 1 || inst[j + 1].tile != t) ranges[2 * t + 1] = j + 1;
    }
}

/* ------------------------------------------------------------------ compositing
 * Pixel (px, py) has centre (px + 0.5, py + 0.5).  Walking the ordered list:
 *   q = (p - m)^T Sigma2D^{-1} (p - m); skip if q > 9 (the 3-sigma ellipse);
 *   alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255;
 *   stop before a Gaussian whose T (1 - alpha) < 1e-4;
 *   C += T alpha c; T *= 1 - alpha.
 * Output C + T bg.  n_contrib = the list positions the pixel reached: the
 * 0-based position of the Gaussian it stopped before, or the list length if
 * it never stopped (every earlier Gaussian that passes both tests was
 * composited, so this and the tests tell which ones were).
 *
 * For the parity protocol, decisions whose FP64 margin is within a relative
 * band are reported ("near"), and a list of positions can be given at which
 * that near decision is taken the other way ("flips"). */

typedef struct {
    int32_t pos;
    int32_t id;
    int32_t clamped;
    double alpha, ex, T, dx, dy;
} or_contrib;

typedef struct {
    const int32_t* flips;
    int32_t nflips;
    double band;
    int32_t* near;
    int32_t n_near, max_near;
} or_decide;

static int is_flip(const or_decide* D, int32_t k) {
    if (!D) return 0;
    for (int32_t j = 0; j < D->nflips; j++)
        if (D->flips[j] == k) return 1;
    return 0;
}

static void note_near(or_decide* D, int32_t k) {
    if (!D || !D->near) return;
    if (D->n_near > 0 && D->near[D->n_near - 1] == k) return;
    if (D->n_near < D->max_near) D->near[D->n_near] = k;
    D->n_near++;
}

/* Returns the number of contributions; rec (optional, sized len) gets them in order. */
static int32_t composite(const or_proj* P, const int32_t* list, int64_t len, double pcx, double pcy,
                         const double bg[3], or_decide* D, double rgb[3], double* Tout, int32_t* nout,
                         or_contrib* rec, int64_t* n_eval) {
    double T = 1.0, C0 = 0.0, C1 = 0.0, C2 = 0.0;
    int32_t n = (int32_t)len, nc = 0;
    const double band = D ? D->band : 0.0;
    for (int64_t k = 0; k < len; k++) {
        const or_proj* g = &P[list[k]];
        const double dx = pcx - g->mean[0], dy = pcy - g->mean[1];
        const double q = g->conic[0] * dx * dx + 2.0 * g->conic[1] * dx * dy + g->conic[2] * dy * dy;
        int flip = is_flip(D, (int32_t)k);
        if (n_eval) (*n_eval)++;
        int pass = q <= OR_Q_MAX;
        if (D && fabs(q - OR_Q_MAX) < band * OR_Q_MAX) {
            note_near(D, (int32_t)k);
            if (flip) { pass = !pass; flip = 0; }
        }
        if (!pass) continue;
        const double ex = exp(-0.5 * q);
        const double araw = g->opacity * ex;
        const int clamped = !(araw < OR_ALPHA_MAX);
        const double alpha = clamped ? OR_ALPHA_MAX : araw;
        pass = alpha >= OR_ALPHA_MIN;
        if (D && fabs(alpha - OR_ALPHA_MIN) < band * OR_ALPHA_MIN) {
            note_near(D, (int32_t)k);
            if (flip) { pass = !pass; flip = 0; }
        }
        if (!pass) continue;
        const double Tn = T * (1.0 - alpha);
        int stop = Tn < OR_T_MIN;
        if (D && fabs(Tn - OR_T_MIN) < band * OR_T_MIN) {
            note_near(D, (int32_t)k);
            if (flip) { stop = !stop; flip = 0; }
        }
        if (stop) {
            n = (int32_t)k;
            break;
        }
        if (rec) {
            rec[nc].pos = (int32_t)k; rec[nc].id = list[k]; rec[nc].clamped = clamped;
            rec[nc].alpha = alpha; rec[nc].ex = ex; rec[nc].T = T; rec[nc].dx = dx; rec[nc].dy = dy;
        }
        nc++;
        C0 += T * alpha * g->color[0];
        C1 += T * alpha * g->color[1];
        C2 += T * alpha * g->color[2];
        T = Tn;
    }
    rgb[0] = C0 + T * bg[0];
    rgb[1] = C1 + T * bg[1];
    rgb[2] = C2 + T * bg[2];
    *Tout = T;
    *nout = n;
    return nc;
}

static void tile_geom(const or_camera* cam, int32_t tw, int32_t th, int32_t* TX, int32_t* TY) {
    *TX = (cam->width + tw - 1) / tw;
    *TY = (cam->height + th - 1) / th;
}

/* Tiled render of one view from the sorted instance ids and per-tile ranges.
 * image is [3][H][W]; counts (optional) gets {pairs evaluated, pairs composited}. */
void or_render(const or_proj* P, const or_camera* cam, int32_t tw, int32_t th, const int32_t* ids,
               const int64_t* ranges, const double* bg, double* image, double* Tfin, int32_t* ncontrib,
               int64_t* counts) {
    int32_t TX, TY;
    tile_geom(cam, tw, th, &TX, &TY);
    const int64_t H = cam->height, W = cam->width, HW = H * W;
    int64_t ev = 0, co = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ev, co)
    for (int64_t t = 0; t < (int64_t)TX * TY; t++) {
        const int32_t tx = (int32_t)(t % TX), ty = (int32_t)(t / TX);
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        for (int32_t ly = 0; ly < th; ly++)
            for (int32_t lx = 0; lx < tw; lx++) {
                const int64_t x = (int64_t)tx * tw + lx, y = (int64_t)ty * th + ly;
                if (x >= W || y >= H) continue;
                double rgb[3], T;
                int32_t n;
                int64_t ne = 0;
                int32_t nc = composite(P, ids + s, e - s, x + 0.5, y + 0.5, bg, NULL, rgb, &T, &n, NULL, &ne);
                ev += ne;
                co += nc;
                for (int ch = 0; ch < 3; ch++) image[ch * HW + y * W + x] = rgb[ch];
                Tfin[y * W + x] = T;
                ncontrib[y * W + x] = n;
            }
    }
    if (counts) { counts[0] = ev; counts[1] = co; }
}

/* Brute force: every Gaussian that survived the z and det culls, ordered by
 * (depth key, id), visits every pixel; no tiles and no rectangles. */
typedef struct { uint32_t key; int32_t id; } or_kid;
static int kid_cmp(const void* a, const void* b) {
    const or_kid* x = (const or_kid*)a;
    const or_kid* y = (const or_kid*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

void or_render_brute(const or_proj* P, int64_t N, const or_camera* cam, const double* bg, double* image,
                     double* Tfin, int32_t* ncontrib) {
    or_kid* kid = (or_kid*)malloc(sizeof(or_kid) * (size_t)(N ? N : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < N; i++)
        if (P[i].radius > 0) { kid[m].key = P[i].key; kid[m].id = (int32_t)i; m++; }
    qsort(kid, (size_t)m, sizeof(or_kid), kid_cmp);
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    for (int64_t j = 0; j < m; j++) list[j] = kid[j].id;
    const int64_t H = cam->height, W = cam->width, HW = H * W;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < HW; p++) {
        const int64_t x = p % W, y = p / W;
        double rgb[3], T;
        int32_t n;
        composite(P, list, m, x + 0.5, y + 0.5, bg, NULL, rgb, &T, &n, NULL, NULL);
        for (int ch = 0; ch < 3; ch++) image[ch * HW + p] = rgb[ch];
        Tfin[p] = T;
        ncontrib[p] = n;
    }
    free(list);
    free(kid);
}

/* Single pixel with optional flips; near (optional) receives near-decision positions. */
int32_t or_pixel(const or_proj* P, const or_camera* cam, int32_t tw, int32_t th, const int32_t* ids,
                 const int64_t* ranges, const double* bg, int32_t x, int32_t y, const int32_t* flips,
                 int32_t nflips, double band, int32_t* near, int32_t max_near, double* rgb, double* T,
                 int32_t* n) {
    int32_t TX, TY;
    tile_geom(cam, tw, th, &TX, &TY);
    const int64_t t = (int64_t)(y / th) * TX + (x / tw);
    or_decide D = {flips, nflips, band, near, 0, max_near};
    composite(P, ids + ranges[2 * t], ranges[2 * t + 1] - ranges[2 * t], x + 0.5, y + 0.5, bg, &D, rgb, T, n,
              NULL, NULL);
    return D.n_near;
}

/* ------------------------------------------------------------------ loss */

double or_loss_l1(const double* img, const double* target, int64_t n, double* G) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double d = img[i] - target[i];
        s += fabs(d);
        G[i] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)n;
    }
    return s / (double)n;
}

/* ------------------------------------------------------------------ adjoint of compositing
 * Decisions are those of the forward pass (optionally with flips per pixel).
 * Walking the contributions back to front with T_k (transmittance in front of
 * k) and B (colour behind k, starting at bg):
 *   dL/dc_k     = T_k alpha_k G
 *   dL/dalpha_k = sum_ch G_ch T_k (c_k,ch - B_ch);   B <- alpha_k c_k + (1 - alpha_k) B
 * and, where alpha was not clamped, alpha = o e^{-q/2}:
 *   dL/do = dL/dalpha e^{-q/2};  dL/dq = -alpha/2 dL/dalpha;
 *   dq/d(a,b,c) = (dx^2, 2 dx dy, dy^2);  dq/dm = -2 [[a,b],[b,c]] (dx, dy).
 * grad2d[i] = (dm_x, dm_y, da, db, dc, do, dc_r, dc_g, dc_b), summed over pixels. */

void or_backward_view(const or_proj* P, int64_t N, const or_camera* cam, int32_t tw, int32_t th,
                      const int32_t* ids, const int64_t* ranges, const double* bg, const double* G,
                      const int32_t* flip_pix, const int32_t* flip_pos, int32_t n_flip_pix, double band,
                      double* grad2d) {
    int32_t TX, TY;
    tile_geom(cam, tw, th, &TX, &TY);
    const int64_t H = cam->height, W = cam->width, HW = H * W;
    const int64_t T = (int64_t)TX * TY;
    int64_t I_all = 0;
    for (int64_t t = 0; t < T; t++) if (ranges[2 * t + 1] > I_all) I_all = ranges[2 * t + 1];
    double* ig = (double*)calloc((size_t)(I_all ? I_all : 1) * 9, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < T; t++) {
        const int32_t tx = (int32_t)(t % TX), ty = (int32_t)(t / TX);
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        if (e <= s) continue;
        or_contrib* rec = (or_contrib*)malloc(sizeof(or_contrib) * (size_t)(e - s));
        for (int32_t ly = 0; ly < th; ly++)
            for (int32_t lx = 0; lx < tw; lx++) {
                const int64_t x = (int64_t)tx * tw + lx, y = (int64_t)ty * th + ly;
                if (x >= W || y >= H) continue;
                const int64_t p = y * W + x;
                const int32_t* fl = NULL;
                int32_t nfl = 0;
                for (int32_t j = 0; j < n_flip_pix; j++)
                    if (flip_pix[j] == p) {
                        fl = flip_pos + 2 * j;
                        nfl = (fl[1] >= 0) ? 2 : ((fl[0] >= 0) ? 1 : 0);
                        break;
                    }
                or_decide D = {fl, nfl, band, NULL, 0, 0};
                double rgb[3], Tf;
                int32_t n;
                int32_t nc = composite(P, ids + s, e - s, x + 0.5, y + 0.5, bg, nfl ? &D : NULL, rgb, &Tf, &n,
                                       rec, NULL);
                const double g0 = G[p], g1 = G[HW + p], g2 = G[2 * HW + p];
                double B0 = bg[0], B1 = bg[1], B2 = bg[2];
                for (int32_t c = nc - 1; c >= 0; c--) {
                    const or_contrib* r = &rec[c];
                    const or_proj* gp = &P[r->id];
                    double* out = ig + 9 * (s + r->pos);
                    const double Ta = r->T * r->alpha;
                    out[6] += Ta * g0;
                    out[7] += Ta * g1;
                    out[8] += Ta * g2;
                    const double da = r->T * ((g0 * (gp->color[0] - B0) + g1 * (gp->color[1] - B1))
                                              + g2 * (gp->color[2] - B2));
                    B0 = r->alpha * gp->color[0] + (1.0 - r->alpha) * B0;
                    B1 = r->alpha * gp->color[1] + (1.0 - r->alpha) * B1;
                    B2 = r->alpha * gp->color[2] + (1.0 - r->alpha) * B2;
                    if (r->clamped) continue;
                    out[5] += da * r->ex;
                    const double dq = -0.5 * r->alpha * da;
                    const double dx = r->dx, dy = r->dy;
                    out[2] += dq * dx * dx;
                    out[3] += dq * 2.0 * dx * dy;
                    out[4] += dq * dy * dy;
                    out[0] += -dq * 2.0 * (gp->conic[0] * dx + gp->conic[1] * dy);
                    out[1] += -dq * 2.0 * (gp->conic[1] * dx + gp->conic[2] * dy);
                }
            }
        free(rec);
    }
    for (int64_t i = 0; i < 9 * N; i++) grad2d[i] = 0.0;
    for (int64_t t = 0; t < T; t++)
        for (int64_t j = ranges[2 * t]; j < ranges[2 * t + 1]; j++)
            for (int k = 0; k < 9; k++) grad2d[9 * ids[j] + k] += ig[9 * j + k];
    free(ig);
}

/* ------------------------------------------------------------------ adjoint of projection
 * With Q the conic matrix and Ghat = [[da, db/2], [db/2, dc]]:
 *   dL/dSigma2D = -Q Ghat Q;  dL/dSigma_c = J^T (dL/dSigma2D) J;
 *   dL/dJ = 2 (dL/dSigma2D) J Sigma_c;  dL/dSigma = R^T (dL/dSigma_c) R;
 *   dL/dM = 2 (dL/dSigma) M;  M = R(q) diag(s);
 *   dm/dmu_c = J;  dJ/dmu_c from J's closed form;  dL/dmu = R^T dL/dmu_c;
 *   colour: dL/dk_j = Y_j(d) dL/dc (0 where the raw colour was < 0), and the
 *   direction term through (I - d d^T)/|mu - c_w|;
 *   texel chain: l_s via s, q through the normalisation (I - qh qh^T)/|q|,
 *   l_o via o (1 - o).
 * Adds into gP[c][i] ([C][N]) for every valid Gaussian of the view. */

static void project_backward_one(const double* P, int64_t N, int64_t i, int32_t L, const or_camera* cam,
                                 const double* g9, double* gP) {
    or_chain c;
    chain_world(P, N, i, &c);
    if (!chain_camera(cam, &c)) return;
    const double det = c.det;
    const double Q[4] = {c.cp / det, -c.bp / det, -c.bp / det, c.ap / det};
    const double Gh[4] = {g9[2], 0.5 * g9[3], 0.5 * g9[3], g9[4]};
    double QG[4], GS[4];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 2; k++) QG[2 * r + k] = Q[2 * r] * Gh[k] + Q[2 * r + 1] * Gh[2 + k];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 2; k++) GS[2 * r + k] = -(QG[2 * r] * Q[k] + QG[2 * r + 1] * Q[2 + k]);
    /* dL/dSigma_c = J^T GS J */
    double GJ[6];  /* GS J : 2x3 */
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++) GJ[3 * r + k] = GS[2 * r] * c.J[k] + GS[2 * r + 1] * c.J[3 + k];
    double GSc[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) GSc[3 * r + k] = c.J[r] * GJ[k] + c.J[3 + r] * GJ[3 + k];
    /* dL/dJ = 2 GS J Sigma_c */
    double GJm[6];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++)
            GJm[3 * r + k] = 2.0 * (GJ[3 * r] * c.Sc[k] + GJ[3 * r + 1] * c.Sc[3 + k] + GJ[3 * r + 2] * c.Sc[6 + k]);
    /* dL/dSigma = R^T GSc R */
    const double* R = cam->R;
    double tmp[9], GSw[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) tmp[3 * r + k] = GSc[3 * r] * R[k] + GSc[3 * r + 1] * R[3 + k] + GSc[3 * r + 2] * R[6 + k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) GSw[3 * r + k] = R[r] * tmp[k] + R[3 + r] * tmp[3 + k] + R[6 + r] * tmp[6 + k];
    /* dL/dM = 2 GSw M */
    double GM[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++)
            GM[3 * r + k] = 2.0 * (GSw[3 * r] * c.M[k] + GSw[3 * r + 1] * c.M[3 + k] + GSw[3 * r + 2] * c.M[6 + k]);
    double gs[3] = {0, 0, 0}, GR[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            gs[k] += GM[3 * r + k] * c.Rq[3 * r + k];
            GR[3 * r + k] = GM[3 * r + k] * c.s[k];
        }
    /* rotation formula -> unit quaternion */
    const double w = c.qh[0], x = c.qh[1], y = c.qh[2], z = c.qh[3];
    double gq[4];
    gq[0] = 2.0 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    gq[1] = 2.0 * (y * GR[1] + z * GR[2] + y * GR[3] - 2.0 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7]
                   - 2.0 * x * GR[8]);
    gq[2] = 2.0 * (-2.0 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7]
                   - 2.0 * y * GR[8]);
    gq[3] = 2.0 * (-2.0 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.0 * z * GR[4] + y * GR[5] + x * GR[6]
                   + y * GR[7]);
    const double qd = gq[0] * c.qh[0] + gq[1] * c.qh[1] + gq[2] * c.qh[2] + gq[3] * c.qh[3];
    /* mean */
    const double zc = c.zc, z2 = zc * zc, z3 = z2 * zc;
    double gmc[3];
    gmc[0] = c.J[0] * g9[0] + c.J[3] * g9[1];
    gmc[1] = c.J[1] * g9[0] + c.J[4] * g9[1];
    gmc[2] = c.J[2] * g9[0] + c.J[5] * g9[1];
    gmc[0] += GJm[2] * (-cam->fx / z2);
    gmc[1] += GJm[5] * (-cam->fy / z2);
    gmc[2] += GJm[0] * (-cam->fx / z2) + GJm[2] * (2.0 * cam->fx * c.xc / z3)
              + GJm[4] * (-cam->fy / z2) + GJm[5] * (2.0 * cam->fy * c.yc / z3);
    double gmu[3];
    for (int k = 0; k < 3; k++) gmu[k] = R[k] * gmc[0] + R[3 + k] * gmc[1] + R[6 + k] * gmc[2];
    /* colour */
    double cw[3], d[3], Y[16], dY[16][3];
    camera_centre(cam, cw);
    for (int k = 0; k < 3; k++) d[k] = c.mu[k] - cw[k];
    const double dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    for (int k = 0; k < 3; k++) d[k] /= dn;
    sh_eval(d, L, Y, dY);
    const int nb = (L + 1) * (L + 1);
    double gd[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ch++) {
        double raw = 0.0;
        for (int j = 0; j < nb; j++) raw += Y[j] * P[(11 + 3 * j + ch) * N + i];
        raw += 0.5;
        const double gc = raw < 0.0 ? 0.0 : g9[6 + ch];
        for (int j = 0; j < nb; j++) {
            const double kk = P[(11 + 3 * j + ch) * N + i];
            gP[(11 + 3 * j + ch) * N + i] += Y[j] * gc;
            for (int a = 0; a < 3; a++) gd[a] += gc * kk * dY[j][a];
        }
    }
    const double dd = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
    for (int k = 0; k < 3; k++) gmu[k] += (gd[k] - d[k] * dd) / dn;
    for (int k = 0; k < 3; k++) gP[k * N + i] += gmu[k];
    for (int k = 0; k < 3; k++) gP[(3 + k) * N + i] += c.s[k] * gs[k];
    for (int k = 0; k < 4; k++) gP[(6 + k) * N + i] += (gq[k] - c.qh[k] * qd) / c.qn;
    gP[10 * N + i] += g9[5] * c.o * (1.0 - c.o);
}

void or_project_backward(const double* P, int64_t N, int32_t L, const or_camera* cam, const or_proj* pr,
                         const double* grad2d, double* gP) {
    sh_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        if (pr[i].valid) project_backward_one(P, N, i, L, cam, grad2d + 9 * i, gP);
}

/* Texel gradients: dL/datlas[f][c][texel(i)] = D(texel) * gP[f][c][i]; 0 elsewhere. */
void or_scatter(const double* gP, const int32_t* ids, const uint8_t* dyn, int32_t F, int32_t C, int32_t H,
                int32_t W, int64_t N, double* gatlas) {
    const int64_t HW = (int64_t)H * W;
    memset(gatlas, 0, sizeof(double) * (size_t)F * C * HW);
    for (int32_t f = 0; f < F; f++)
        for (int32_t c = 0; c < C; c++)
            for (int64_t i = 0; i < N; i++) {
                double m = dyn ? (double)(dyn[ids[i]] != 0) : 1.0;
                gatlas[((int64_t)f * C + c) * HW + ids[i]] = m * gP[((int64_t)f * C + c) * N + i];
            }
}

/* ------------------------------------------------------------------ frozen-decision finite differences
 * <G, I(theta)> restricted to the pixels whose tile lists hold Gaussian i,
 * with every decision (culls, rectangles, list order, which Gaussians each
 * pixel composites, where it stops, alpha and colour clamps) taken at the
 * unperturbed point and only the values recomputed with parameter ch of
 * Gaussian i moved by +h and -h.  Returns (F(+h) - F(-h)) / (2h) for one view. */

static double frozen_sum(const or_proj* P0, const or_proj* gi, int64_t i, const or_camera* cam, int32_t tw,
                         int32_t th, const int32_t* ids, const int64_t* ranges, const double* bg,
                         const double* G, or_contrib* rec) {
    int32_t TX, TY;
    tile_geom(cam, tw, th, &TX, &TY);
    const int64_t H = cam->height, W = cam->width, HW = H * W;
    const or_proj* p0 = &P0[i];
    double acc = 0.0;
    for (int32_t ty = p0->rect[1]; ty <= p0->rect[3]; ty++)
        for (int32_t tx = p0->rect[0]; tx <= p0->rect[2]; tx++) {
            const int64_t t = (int64_t)ty * TX + tx;
            const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
            for (int32_t ly = 0; ly < th; ly++)
                for (int32_t lx = 0; lx < tw; lx++) {
                    const int64_t x = (int64_t)tx * tw + lx, y = (int64_t)ty * th + ly;
                    if (x >= W || y >= H) continue;
                    double rgb[3], T;
                    int32_t n;
                    int32_t nc = composite(P0, ids + s, e - s, x + 0.5, y + 0.5, bg, NULL, rgb, &T, &n, rec, NULL);
                    int hit = 0;
                    for (int32_t c = 0; c < nc; c++) hit |= (rec[c].id == (int32_t)i);
                    if (!hit) continue;
                    /* re-evaluate with frozen decisions and perturbed values for i */
                    double Tv = 1.0, C3[3] = {0, 0, 0};
                    for (int32_t c = 0; c < nc; c++) {
                        const or_contrib* r = &rec[c];
                        double alpha = r->alpha;
                        const double* col = P0[r->id].color;
                        double colp[3];
                        if (r->id == (int32_t)i) {
                            const double dx = x + 0.5 - gi->mean[0], dy = y + 0.5 - gi->mean[1];
                            const double q = gi->conic[0] * dx * dx + 2.0 * gi->conic[1] * dx * dy
                                             + gi->conic[2] * dy * dy;
                            alpha = r->clamped ? OR_ALPHA_MAX : gi->opacity * exp(-0.5 * q);
                            for (int k = 0; k < 3; k++)
                                colp[k] = p0->color_raw[k] < 0.0 ? 0.0 : gi->color_raw[k];
                            col = colp;
                        }
                        for (int k = 0; k < 3; k++) C3[k] += Tv * alpha * col[k];
                        Tv *= 1.0 - alpha;
                    }
                    for (int k = 0; k < 3; k++) C3[k] += Tv * bg[k];
                    acc += G[y * W + x] * C3[0] + G[HW + y * W + x] * C3[1] + G[2 * HW + y * W + x] * C3[2];
                }
        }
    return acc;
}

double or_fd_frozen(const double* P, int64_t N, int32_t C, int32_t L, const or_camera* cam, int32_t tw,
                    int32_t th, const or_proj* P0, const int32_t* ids, const int64_t* ranges, const double* bg,
                    const double* G, int64_t i, int32_t ch, double h) {
    sh_init();
    if (!P0[i].valid) return 0.0;
    int64_t maxlen = 0;
    int32_t TX, TY;
    tile_geom(cam, tw, th, &TX, &TY);
    for (int64_t t = 0; t < (int64_t)TX * TY; t++)
        if (ranges[2 * t + 1] - ranges[2 * t] > maxlen) maxlen = ranges[2 * t + 1] - ranges[2 * t];
    or_contrib* rec = (or_contrib*)malloc(sizeof(or_contrib) * (size_t)(maxlen ? maxlen : 1));
    /* one-Gaussian copy of the parameter planes */
    double* Pi = (double*)malloc(sizeof(double) * (size_t)C);
    for (int32_t c = 0; c < C; c++) Pi[c] = P[(int64_t)c * N + i];
    or_proj gp, gm;
    const double v0 = Pi[ch];
    Pi[ch] = v0 + h;
    project_one(Pi, 1, 0, L, cam, tw, th, &gp);
    Pi[ch] = v0 - h;
    project_one(Pi, 1, 0, L, cam, tw, th, &gm);
    double fp = frozen_sum(P0, &gp, i, cam, tw, th, ids, ranges, bg, G, rec);
    double fm = frozen_sum(P0, &gm, i, cam, tw, th, ids, ranges, bg, G, rec);
    free(Pi);
    free(rec);
    return (fp - fm) / (2.0 * h);
}

/* ------------------------------------------------------------------ Adam
 * Textbook Adam (Kingma & Ba) with bias correction at global step t, applied
 * only where visible[e] != 0 ("sparse": texels whose Gaussian was drawn in at
 * least one view this step). */
void or_adam(double* p, const double* g, double* m, double* v, const uint8_t* visible, int64_t n, double lr,
             double b1, double b2, double eps, int32_t t) {
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t e = 0; e < n; e++) {
        if (!visible[e]) continue;
        m[e] = b1 * m[e] + (1.0 - b1) * g[e];
        v[e] = b2 * v[e] + (1.0 - b2) * g[e] * g[e];
        const double mh = m[e] / c1, vh = v[e] / c2;
        p[e] = p[e] - lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------ UV pruning
 * UV-based pruning (Sec. 4.2 "UV-Based Pruning", with the UV projection
 * equation of Sec. 3): a Gaussian's position in spherical coordinates
 * (rho, theta = atan2(y, x), phi = acos(z / rho)) gives the UV pixel
 * u = floor((pi + theta) / (2 pi) M), v = floor(phi / pi N) of an M x N map.
 * theta = pi (the direction of -pi) wraps to u = 0; phi = pi stays in the
 * last row; rho = 0 has no direction and is invalid.  Valid UV projection:
 * when expected (the pixel v M + u of the texel that stores the Gaussian) is
 * given, a Gaussian that maps elsewhere is invalid.  Max-K: among the valid
 * Gaussians of a pixel, the K of highest opacity are kept (ranked by the
 * logit, which orders like the opacity; ties by ascending id).
 *   uv    int32 [N] out: v M + u, -1 if invalid
 *   rank  int32 [N] out: rank inside the pixel, -1 if invalid
 *   keep  uint8 [N] out */
typedef struct {
    int32_t key, id;
    double logit;
} or_uvrec;

static int uvrec_cmp(const void* pa, const void* pb) {
    const or_uvrec* a = (const or_uvrec*)pa;
    const or_uvrec* b = (const or_uvrec*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->logit != b->logit) return a->logit > b->logit ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

void or_uv_prune(const double* P, int64_t N, int32_t M, int32_t Nv, int32_t K, const int32_t* expected,
                 int32_t* uv, int32_t* rank, uint8_t* keep) {
    or_uvrec* r = (or_uvrec*)malloc(sizeof(or_uvrec) * (size_t)(N > 0 ? N : 1));
    int64_t n = 0;
    for (int64_t i = 0; i < N; i++) {
        const double x = P[0 * N + i], y = P[1 * N + i], z = P[2 * N + i];
        const double rho = sqrt((x * x + y * y) + z * z);
        uv[i] = -1;
        rank[i] = -1;
        keep[i] = 0;
        if (!(rho > 0.0)) continue;
        const double theta = atan2(y, x);
        double c = z / rho;
        c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
        const double phi = acos(c);
        int64_t u = (int64_t)floor((3.141592653589793 + theta) / (2.0 * 3.141592653589793) * (double)M);
        int64_t v = (int64_t)floor(phi / 3.141592653589793 * (double)Nv);
        if (u >= M) u -= M;
        if (v >= Nv) v = Nv - 1;
        const int32_t key = (int32_t)(v * M + u);
        if (expected && expected[i] != key) continue;
        uv[i] = key;
        r[n].key = key;
        r[n].id = (int32_t)i;
        r[n].logit = P[10 * N + i];
        n++;
    }
    qsort(r, (size_t)n, sizeof(or_uvrec), uvrec_cmp);
    for (int64_t j = 0, start = 0; j < n; j++) {
        if (j > 0 && r[j].key != r[j - 1].key) start = j;
        rank[r[j].id] = (int32_t)(j - start);
        keep[r[j].id] = (j - start) < K;
    }
    free(r);
}

/* ------------------------------------------------------------------ SSIM
 * Structural similarity of the photometric objective (Sec. 4.2
 * "Objective"; the paper names SSIM without its parameters, read here as
 * the usual definition): per channel plane, local statistics under an
 * 11 x 11 Gaussian window (sigma 1.5, weights normalised to sum 1) with zero
 * padding outside the image,
 *   a = w * x, b = w * y, c = w * x^2, d = w * y^2, e = w * x y,
 *   S = (2 a b + C1) (2 (e - a b) + C2) / ((a^2 + b^2 + C1) ((c - a^2) + (d - b^2) + C2)),
 * C1 = 0.01^2, C2 = 0.03^2 (data range 1).  Returns the sum of S over the
 * plane (smap, if given, receives S per pixel); grad (or NULL) receives
 * d(sum S)/dx, by the chain rule through the
 * five window sums:  dS/da = 2 b (N2 - N1) / (D1 D2) - S (2 a / D1 - 2 a / D2),
 * dS/dc = -S / D2, dS/de = 2 N1 / (D1 D2), and each window sum's adjoint is
 * the same window correlation (the window is symmetric). */
#define OR_SSIM_R 5
#define OR_SSIM_C1 (0.01 * 0.01)
#define OR_SSIM_C2 (0.03 * 0.03)

static void ssim_window(double w[2 * OR_SSIM_R + 1]) {
    double sum = 0.0;
    for (int k = 0; k <= 2 * OR_SSIM_R; k++) {
        const double t = (double)(k - OR_SSIM_R);
        w[k] = exp(-(t * t) / (2.0 * 1.5 * 1.5));
        sum += w[k];
    }
    for (int k = 0; k <= 2 * OR_SSIM_R; k++) w[k] /= sum;
}

double or_ssim(const double* x, const double* y, int32_t H, int32_t W, double* grad, double* smap) {
    const int R = OR_SSIM_R;
    double w[2 * OR_SSIM_R + 1];
    ssim_window(w);
    const int64_t n = (int64_t)H * W;
    double* pa = grad ? (double*)calloc((size_t)n, sizeof(double)) : NULL;
    double* pc = grad ? (double*)calloc((size_t)n, sizeof(double)) : NULL;
    double* pe = grad ? (double*)calloc((size_t)n, sizeof(double)) : NULL;
    double total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int32_t py = 0; py < H; py++)
        for (int32_t px = 0; px < W; px++) {
            double a = 0.0, b = 0.0, c = 0.0, d = 0.0, e = 0.0;
            for (int dy = -R; dy <= R; dy++)
                for (int dx = -R; dx <= R; dx++) {
                    const int32_t qy = py + dy, qx = px + dx;
                    if (qy < 0 || qy >= H || qx < 0 || qx >= W) continue;   /* zero padding */
                    const double wt = w[dy + R] * w[dx + R];
                    const double xv = x[(int64_t)qy * W + qx], yv = y[(int64_t)qy * W + qx];
                    a += wt * xv;
                    b += wt * yv;
                    c += wt * xv * xv;
                    d += wt * yv * yv;
                    e += wt * xv * yv;
                }
            const double N1 = 2.0 * a * b + OR_SSIM_C1, N2 = 2.0 * (e - a * b) + OR_SSIM_C2;
            const double D1 = a * a + b * b + OR_SSIM_C1, D2 = (c - a * a) + (d - b * b) + OR_SSIM_C2;
            const double S = (N1 * N2) / (D1 * D2);
            total += S;
            if (smap) smap[(int64_t)py * W + px] = S;
            if (grad) {
                const int64_t p = (int64_t)py * W + px;
                pa[p] = 2.0 * b * (N2 - N1) / (D1 * D2) - S * (2.0 * a / D1 - 2.0 * a / D2);
                pc[p] = -S / D2;
                pe[p] = 2.0 * N1 / (D1 * D2);
            }
        }
    if (grad) {
#pragma omp parallel for schedule(static)
        for (int32_t qy = 0; qy < H; qy++)
            for (int32_t qx = 0; qx < W; qx++) {
                double A = 0.0, Cc = 0.0, E = 0.0;
                for (int dy = -R; dy <= R; dy++)
                    for (int dx = -R; dx <= R; dx++) {
                        const int32_t py = qy + dy, px = qx + dx;
                        if (py < 0 || py >= H || px < 0 || px >= W) continue;
                        const double wt = w[dy + R] * w[dx + R];
                        const int64_t p = (int64_t)py * W + px;
                        A += wt * pa[p];
                        Cc += wt * pc[p];
                        E += wt * pe[p];
                    }
                const int64_t q = (int64_t)qy * W + qx;
                grad[q] = A + 2.0 * x[q] * Cc + y[q] * E;
            }
        free(pa);
        free(pc);
        free(pe);
    }
    return total;
}

/* ------------------------------------------------------------------ regularisers
 * Scale and opacity regularisers of the objective (Sec. 4.2 "Objective"),
 * over the Gaussians of every frame, or only the dynamic ones (dyn[f N + i]
 * != 0) when dyn is given:
 *   L_scale   = mean_i max(0, max_k s_ik - s_max)^2,  s = exp(l_s),
 *   L_opacity = mean_i o_i (1 - o_i),                 o = sigmoid(l_o).
 * Their gradients with respect to the texel channels (l_s through exp, l_o
 * through the sigmoid) are written to grad [F][C][N] (channels 3-5 and 10;
 * zero elsewhere) as dL_scale and dL_opacity scaled by w_scale, w_opacity.
 * Writes the two means to out[0], out[1]; returns the number averaged. */
int64_t or_regularisers(const double* P, int32_t F, int32_t C, int64_t N, const uint8_t* dyn, double s_max,
                        double w_scale, double w_opacity, double* grad, double* out) {
    int64_t n = 0;
    for (int64_t g = 0; g < (int64_t)F * N; g++)
        if (!dyn || dyn[g]) n++;
    memset(grad, 0, sizeof(double) * (size_t)((int64_t)F * C * N));
    double ls = 0.0, lo = 0.0;
    for (int32_t f = 0; f < F; f++)
        for (int64_t i = 0; i < N; i++) {
            if (dyn && !dyn[(int64_t)f * N + i]) continue;
            const double* Pf = P + (int64_t)f * C * N;
            double* Gf = grad + (int64_t)f * C * N;
            int kmax = 0;
            double smax = exp(Pf[3 * N + i]);
            for (int k = 1; k < 3; k++) {
                const double sk = exp(Pf[(3 + k) * N + i]);
                if (sk > smax) { smax = sk; kmax = k; }
            }
            const double h = smax > s_max ? smax - s_max : 0.0;
            ls += h * h;
            Gf[(3 + kmax) * N + i] = w_scale * (2.0 * h * smax) / (double)n;   /* d/dl of exp(l) is exp(l) */
            const double o = 1.0 / (1.0 + exp(-Pf[10 * N + i]));
            lo += o * (1.0 - o);
            Gf[10 * N + i] = w_opacity * ((1.0 - 2.0 * o) * o * (1.0 - o)) / (double)n;
        }
    out[0] = n ? ls / (double)n : 0.0;
    out[1] = n ? lo / (double)n : 0.0;
    return n;
}

/* ------------------------------------------------------------------ flow masking
 * Covariance-aware flow masking (Sec. 4.2 "Covariance-Aware Gaussian
 * Masking", Algorithm 1): project the Gaussian with the EWA chain above
 * (same culls; a culled projection leaves it static for this camera), take
 * the sampling radius r = ceil(3 sqrt(lambda_max)), and scan the pixels whose
 * centre (x + 0.5, y + 0.5) lies within r of the mean on both axes, inside
 * the image; the Gaussian is dynamic for the camera when one of them has
 * d^2 = q <= 9 (FP64, the conic of the projection) and a non-zero flow mask.
 * D is OR-ed in place, so calling this for each camera of a frame gives the
 * paper's OR across cameras.
 *   mask  uint8 [H][W] of this camera;  D  uint8 [N] in/out */
static double q_at(double A, double B, double C, double X, double Y) {
    return (A * X * X + 2.0 * B * X * Y) + C * Y * Y;
}

void or_flow_mask(const double* P, int64_t N, int32_t L, const or_camera* cam, const uint8_t* mask,
                  uint8_t* D) {
    const int32_t W = cam->width, H = cam->height;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; i++) {
        if (D[i]) continue;
        or_proj o;
        project_one(P, N, i, L, cam, 16, 16, &o);
        if (o.radius <= 0) continue;   /* culled: z or det */
        const double r = (double)o.radius;
        const double x0 = fmax(0.0, ceil(o.mean[0] - r - 0.5)), x1 = fmin((double)(W - 1), floor(o.mean[0] + r - 0.5));
        const double y0 = fmax(0.0, ceil(o.mean[1] - r - 0.5)), y1 = fmin((double)(H - 1), floor(o.mean[1] + r - 0.5));
        int hit = 0;
        for (double y = y0; y <= y1 && !hit; y += 1.0)
            for (double x = x0; x <= x1; x += 1.0) {
                if (!mask[(int64_t)y * W + (int64_t)x]) continue;
                const double dx = (x + 0.5) - o.mean[0], dy = (y + 0.5) - o.mean[1];
                if (q_at(o.conic[0], o.conic[1], o.conic[2], dx, dy) <= 9.0) {
                    hit = 1;
                    break;
                }
            }
        if (hit) D[i] = 1;
    }
}

/* ------------------------------------------------------------------ LPO fake quantiser
 * Low-precision optimisation (Sec. 4.3 LPO paragraph; supplementary,
 * low-precision training): the renderer consumes a uniform K-bit proxy of
 * the texel values, gradients pass straight through to the FP32 master
 * values, and the scale comes from a per-channel min/max normalisation (the
 * video-coding section normalises each channel by its min/max).  Reading:
 * per channel c with K = bits[c] > 0, lo / hi = min / max over the occupied
 * texels of every frame, levels = 2^K - 1, delta = (hi - lo) / levels,
 * code = clamp(rint((v - lo) / delta), 0, levels), proxy = lo + code delta.
 * The code is an integer decided by floating point, so it is computed in the
 * precision of the texels, FP32, each operation rounded once (no
 * contraction), ties to even; delta = 0 gives code 0 and proxy lo.
 * Unoccupied texels and channels with bits[c] = 0 are copied unchanged.
 *   range  float [C][2] out (lo, hi; 0, 0 for unquantised channels)
 *   codes  uint16 [F][C][H][W] out or NULL (0 where nothing is quantised) */
void or_fake_quant(const float* atlas, const uint8_t* occ, int32_t F, int32_t C, int32_t H, int32_t W,
                   const int32_t* bits, float* range, float* out, uint16_t* codes) {
    const int64_t HW = (int64_t)H * W;
    memcpy(out, atlas, sizeof(float) * (size_t)((int64_t)F * C * HW));
    if (codes) memset(codes, 0, sizeof(uint16_t) * (size_t)((int64_t)F * C * HW));
    for (int32_t c = 0; c < C; c++) {
        range[2 * c] = range[2 * c + 1] = 0.0f;
        if (bits[c] <= 0) continue;
        float lo = INFINITY, hi = -INFINITY;
        for (int32_t f = 0; f < F; f++)
            for (int64_t p = 0; p < HW; p++)
                if (occ[p]) {
                    const float v = atlas[((int64_t)f * C + c) * HW + p];
                    lo = fminf(lo, v);
                    hi = fmaxf(hi, v);
                }
        if (lo > hi) continue;   /* no occupied texel */
        range[2 * c] = lo;
        range[2 * c + 1] = hi;
        const float levels = (float)((1 << bits[c]) - 1);
        const float delta = (hi - lo) / levels;
        for (int32_t f = 0; f < F; f++)
            for (int64_t p = 0; p < HW; p++) {
                if (!occ[p]) continue;
                const int64_t e = ((int64_t)f * C + c) * HW + p;
                float k = 0.0f;
                if (delta > 0.0f) {
                    const float d = atlas[e] - lo;
                    k = rintf(d / delta);
                    k = fminf(fmaxf(k, 0.0f), levels);
                }
                const float step = k * delta;
                out[e] = lo + step;
                if (codes) codes[e] = (uint16_t)k;
            }
    }
}

void or_set_num_threads(int32_t n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int32_t or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
