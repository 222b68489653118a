/*
 * FP64 CPU oracle for the differentiable bitmap-primitive rasteriser of DiffBMP
 * (arXiv 2602.22625, Sec. 3.1 and Supplementary Sec. S1).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg load or call this library. It shares no code with the GPU path and must never be used to
 * produce a product result.
 *
 * It computes the plain definition: every pixel walks every primitive in index order (index 0 is
 * the front layer), exactly the structure of the naive baseline (Supp. Alg. 3), with no tiling,
 * no binning and no culling beyond the exact zero of the bilinear sampler outside the bitmap.
 *
 * Readings of points the paper leaves open (listed with reasons in the design notes):
 *   - pixel (px, py) sits at canvas point (x, y) = (px, py), origin top-left, y down;
 *   - texels outside the bitmap read as 0 (zero padding of the bilinear sampler, Alg. 3 uses
 *     grid_sample whose default padding is zeros);
 *   - the background b is composited behind all layers: I = C + T_N b (Eq. 8 form);
 *   - scale is learned as log s;  gradients are reported w.r.t. log s;
 *   - at an exactly integer U or V the floor cell is used (one-sided derivative);
 *   - no epsilon skip, no per-pixel primitive cap, no early termination.
 *
 * Parameter row (8 doubles per primitive): x, y, log_s, theta, nu, c_r, c_g, c_b.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double alpha;   /* alpha_k at this pixel (Eq. 3) */
    double M;       /* bilinear template value (Supp. Eqs. S1-S3) */
    double MU, MV;  /* dM/dU, dM/dV on the floor cell */
    double u, v;    /* normalised primitive coordinates (Eq. 1) */
} pair_eval;

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

static double texel(const double *bm, int Hb, int Wb, int r, int c)
{
    if (r < 0 || r >= Hb || c < 0 || c >= Wb) return 0.0;  /* zero padding */
    return bm[(size_t)r * Wb + c];
}

/* Evaluates primitive p at canvas point (x, y). Returns 0 when all four lattice neighbours lie
 * outside the bitmap: there M and both its partial derivatives are exactly zero. */
static int eval_pair(const double *p, const double *bm, int Hb, int Wb, double alpha_max,
                     double x, double y, pair_eval *e)
{
    const double s = exp(p[2]);
    const double ct = cos(p[3]), st = sin(p[3]);
    const double dx = x - p[0], dy = y - p[1];
    /* Eq. (1): rotate by R(theta) and divide by the scale */
    const double u = (ct * dx + st * dy) / s;
    const double v = (-st * dx + ct * dy) / s;
    /* Eq. (2): normalised [-1,1] -> bitmap lattice [0, W-1] x [0, H-1] */
    const double U = (u + 1.0) / 2.0 * (Wb - 1);
    const double V = (v + 1.0) / 2.0 * (Hb - 1);
    const double u0 = floor(U), v0 = floor(V);
    if (u0 < -1.0 || u0 > (double)(Wb - 1) || v0 < -1.0 || v0 > (double)(Hb - 1)) return 0;
    const int iu = (int)u0, iv = (int)v0;
    const double wu = U - u0, wv = V - v0;
    /* Supp. Eq. (S2): the four neighbours p = [P[v0,u0], P[v0,u0+1], P[v0+1,u0], P[v0+1,u0+1]] */
    const double p00 = texel(bm, Hb, Wb, iv, iu);
    const double p01 = texel(bm, Hb, Wb, iv, iu + 1);
    const double p10 = texel(bm, Hb, Wb, iv + 1, iu);
    const double p11 = texel(bm, Hb, Wb, iv + 1, iu + 1);
    /* Supp. Eqs. (S1), (S3): M = w^T p */
    e->M = (1.0 - wu) * (1.0 - wv) * p00 + wu * (1.0 - wv) * p01
         + (1.0 - wu) * wv * p10 + wu * wv * p11;
    e->MU = (1.0 - wv) * (p01 - p00) + wv * (p11 - p10);
    e->MV = (1.0 - wu) * (p10 - p00) + wu * (p11 - p01);
    e->u = u;
    e->v = v;
    /* Eq. (3) */
    e->alpha = alpha_max * sigmoid(p[4]) * e->M;
    return 1;
}

static const double *bg_at(const double *bg, int bg_per_pixel, int H, int W, int px, int py,
                           double out[3])
{
    if (bg_per_pixel) {
        const size_t plane = (size_t)H * W, o = (size_t)py * W + px;
        out[0] = bg[o]; out[1] = bg[plane + o]; out[2] = bg[2 * plane + o];
    } else {
        out[0] = bg[0]; out[1] = bg[1]; out[2] = bg[2];
    }
    return out;
}

/*
 * Forward (Eqs. 3-5 with the background term): image [3, h, w] and alpha [h, w] = 1 - T_N of
 * the crop window [x0, x0+w) x [y0, y0+h) of an H x W canvas.
 * atlas: [B, Hb, Wb] row-major; idx[k] in [0, B) selects primitive k's bitmap.
 * bg: 3 values, or [3, H, W] when bg_per_pixel != 0.
 * Returns 0, or -1 on invalid arguments (bad crop or an atlas index out of range).
 */
int oracle_render(int N, const double *params, const int *idx, const double *atlas, int B,
                  int Hb, int Wb, int H, int W, const double *bg, int bg_per_pixel,
                  double alpha_max, int x0, int y0, int w, int h, double *image, double *alpha,
                  int nthreads)
{
    if (x0 < 0 || y0 < 0 || w < 0 || h < 0 || x0 + w > W || y0 + h > H || Hb < 2 || Wb < 2)
        return -1;
    for (int k = 0; k < N; ++k)
        if (idx[k] < 0 || idx[k] >= B) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const size_t plane = (size_t)h * w;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < h; ++r) {
        for (int c = 0; c < w; ++c) {
            const int px = x0 + c, py = y0 + r;
            double T = 1.0, C[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < N; ++k) {  /* front to back: index 0 has T_0 = 1 (Eq. 4) */
                const double *p = params + (size_t)k * 8;
                const double *bm = atlas + (size_t)idx[k] * Hb * Wb;
                pair_eval e;
                if (!eval_pair(p, bm, Hb, Wb, alpha_max, (double)px, (double)py, &e)) continue;
                for (int j = 0; j < 3; ++j) C[j] += T * e.alpha * sigmoid(p[5 + j]);  /* Eq. 5 */
                T *= (1.0 - e.alpha);                                                  /* Eq. 4 */
            }
            double b[3];
            bg_at(bg, bg_per_pixel, H, W, px, py, b);
            const size_t o = (size_t)r * w + c;
            for (int j = 0; j < 3; ++j) image[j * plane + o] = C[j] + T * b[j];
            if (alpha) alpha[o] = 1.0 - T;
        }
    }
    return 0;
}

/*
 * Backward: dparams [N, 8] (overwritten) = sum over the crop's pixels of the chain rule of
 * Eq. (7) and Supp. Eqs. (S4)-(S5), given gI = dL/dI [3, h, w] and gA = dL/dA [h, w] (may be
 * NULL) for the crop window. The suffix sum S_j / (1 - alpha_k) of Eq. (S5) is carried as
 * T_k * (G_j - B b_j) through the back-to-front recurrences
 *     G <- alpha_k c_k + (1 - alpha_k) G   (starting at the background b),
 *     B <- (1 - alpha_k) B                  (starting at 1),
 * which is the same quantity written without the division, so alpha_k = 1 is allowed.
 */
int oracle_render_backward(int N, const double *params, const int *idx, const double *atlas,
                           int B, int Hb, int Wb, int H, int W, const double *bg,
                           int bg_per_pixel, double alpha_max, int x0, int y0, int w, int h,
                           const double *gI, const double *gA, double *dparams, int nthreads)
{
    if (x0 < 0 || y0 < 0 || w < 0 || h < 0 || x0 + w > W || y0 + h > H || Hb < 2 || Wb < 2)
        return -1;
    for (int k = 0; k < N; ++k)
        if (idx[k] < 0 || idx[k] >= B) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int nt = omp_get_max_threads();
#else
    (void)nthreads;
    const int nt = 1;
#endif
    double *acc = (double *)calloc((size_t)nt * N * 8 + 1, sizeof(double));
    if (!acc) return -2;
    const size_t plane = (size_t)h * w;
    const double half_w = 0.5 * (Wb - 1), half_h = 0.5 * (Hb - 1);  /* dU/du, dV/dv (Eq. 2) */

#pragma omp parallel
    {
#ifdef _OPENMP
        const int tid = omp_get_thread_num();
#else
        const int tid = 0;
#endif
        double *g = acc + (size_t)tid * N * 8;
        int *ks = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
        double *Ts = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        pair_eval *ev = (pair_eval *)malloc(sizeof(pair_eval) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(static)
        for (int r = 0; r < h; ++r) {
            for (int c = 0; c < w; ++c) {
                const int px = x0 + c, py = y0 + r;
                const size_t o = (size_t)r * w + c;
                /* forward walk, recording the layers that touch this pixel */
                int n = 0;
                double T = 1.0;
                for (int k = 0; k < N; ++k) {
                    const double *p = params + (size_t)k * 8;
                    const double *bm = atlas + (size_t)idx[k] * Hb * Wb;
                    if (!eval_pair(p, bm, Hb, Wb, alpha_max, (double)px, (double)py, &ev[n]))
                        continue;
                    ks[n] = k;
                    Ts[n] = T;            /* T_k, transmittance in front of layer k */
                    T *= (1.0 - ev[n].alpha);
                    ++n;
                }
                double G[3], gi[3];
                bg_at(bg, bg_per_pixel, H, W, px, py, G);
                for (int j = 0; j < 3; ++j) gi[j] = gI[j * plane + o];
                const double ga = gA ? gA[o] : 0.0;
                double Bk = 1.0;
                for (int m = n - 1; m >= 0; --m) {
                    const int k = ks[m];
                    const double *p = params + (size_t)k * 8;
                    const pair_eval *e = &ev[m];
                    const double Tk = Ts[m], a = e->alpha;
                    double chat[3];
                    for (int j = 0; j < 3; ++j) chat[j] = sigmoid(p[5 + j]);
                    /* dL/dalpha_k (Supp. Eq. S5) */
                    double dal = ga * Bk;
                    for (int j = 0; j < 3; ++j) dal += gi[j] * (chat[j] - G[j]);
                    dal *= Tk;
                    double *gk = g + (size_t)k * 8;
                    /* colour logits (Supp. Eq. S4) */
                    for (int j = 0; j < 3; ++j)
                        gk[5 + j] += gi[j] * Tk * a * chat[j] * (1.0 - chat[j]);
                    /* opacity logit through Eq. (3) */
                    const double sg = sigmoid(p[4]);
                    gk[4] += dal * alpha_max * sg * (1.0 - sg) * e->M;
                    /* geometry through M -> (U, V) -> (u, v) -> (x_k, y_k, log s_k, theta_k), Eq. (7) */
                    const double dM = dal * alpha_max * sg;
                    const double du = dM * e->MU * half_w, dv = dM * e->MV * half_h;
                    const double s = exp(p[2]), ct = cos(p[3]), st = sin(p[3]);
                    gk[0] += du * (-ct / s) + dv * (st / s);
                    gk[1] += du * (-st / s) + dv * (-ct / s);
                    gk[2] += -(du * e->u + dv * e->v);
                    gk[3] += du * e->v - dv * e->u;
                    for (int j = 0; j < 3; ++j) G[j] = a * chat[j] + (1.0 - a) * G[j];
                    Bk *= (1.0 - a);
                }
            }
        }
        free(ks);
        free(Ts);
        free(ev);
    }
    memset(dparams, 0, sizeof(double) * (size_t)N * 8);
    for (int t = 0; t < nt; ++t)  /* fixed thread order: deterministic for a given thread count */
        for (size_t q = 0; q < (size_t)N * 8; ++q) dparams[q] += acc[(size_t)t * N * 8 + q];
    free(acc);
    return 0;
}

/*
 * Per-pixel trace for invariant checks: the layers that touch pixel (px, py), in front-to-back
 * order, with alpha_k and the transmittance T_k in front of each. Writes at most `cap` entries
 * and returns the number of touching layers (or -1 on bad arguments); *T_final = T_N.
 */
int oracle_pixel_trace(int N, const double *params, const int *idx, const double *atlas, int B,
                       int Hb, int Wb, double alpha_max, int px, int py, int cap, int *ks,
                       double *alphas, double *Ts, double *T_final)
{
    if (Hb < 2 || Wb < 2) return -1;
    int n = 0;
    double T = 1.0;
    for (int k = 0; k < N; ++k) {
        if (idx[k] < 0 || idx[k] >= B) return -1;
        const double *p = params + (size_t)k * 8;
        const double *bm = atlas + (size_t)idx[k] * Hb * Wb;
        pair_eval e;
        if (!eval_pair(p, bm, Hb, Wb, alpha_max, (double)px, (double)py, &e)) continue;
        if (n < cap) {
            ks[n] = k;
            alphas[n] = e.alpha;
            Ts[n] = T;
        }
        T *= (1.0 - e.alpha);
        ++n;
    }
    *T_final = T;
    return n;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Exact number of (pixel, primitive) pairs of the crop window where the primitive's bilinear
 * sampler reads at least one lattice point inside its bitmap (the pairs the method evaluates).
 */
long long oracle_support_pairs(int N, const double *params, const int *idx, int B, int Hb,
                               int Wb, int x0, int y0, int w, int h, int nthreads)
{
    (void)B;
    (void)idx;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    long long total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int r = 0; r < h; ++r) {
        for (int c = 0; c < w; ++c) {
            const double x = x0 + c, y = y0 + r;
            for (int k = 0; k < N; ++k) {
                const double *p = params + (size_t)k * 8;
                const double s = exp(p[2]), ct = cos(p[3]), st = sin(p[3]);
                const double dx = x - p[0], dy = y - p[1];
                const double U = ((ct * dx + st * dy) / s + 1.0) / 2.0 * (Wb - 1);
                const double V = ((-st * dx + ct * dy) / s + 1.0) / 2.0 * (Hb - 1);
                const double u0 = floor(U), v0 = floor(V);
                if (u0 >= -1.0 && u0 <= (double)(Wb - 1) && v0 >= -1.0 && v0 <= (double)(Hb - 1))
                    ++total;
            }
        }
    }
    return total;
}
