/*
 * FP64 brute-force oracle of the point-cloud rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it; the product path never does.
 *
 * Paper, Section 3.3 ("Differentiable point cloud renderer"): every point is
 * splatted to a disc in screen space, and the rasterizer returns for each
 * pixel the K points nearest along z whose discs cover the pixel, with their
 * depth and squared xy distance to the pixel centre.  Readings (the paper
 * leaves them open): pixel centres as for meshes (x = 1 - (2c+1)/W,
 * y = 1 - (2r+1)/H); a point covers a pixel iff the squared xy distance is
 * strictly below radius^2 and its z is not negative; ties in z are broken by
 * the packed point index; empty slots hold -1 in idx, zbuf and dists.
 *
 * Method: every pixel tests every point of its image's cloud, the hits are
 * sorted by (z, index) and the first K kept.  The backward is the analytic
 * derivative of L = <gz, zbuf> + <gd, dists> with the choice of points held
 * fixed: zbuf_k = z_p and dists_k = (x_p - px)^2 + (y_p - py)^2, so
 * dL/dz_p += gz_k and dL/d(x_p, y_p) += 2 gd_k (x_p - px, y_p - py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PT_TAU 1e-6 /* decision margin in linear NDC units */

static void pt_pixel_center(int64_t r, int64_t c, int H, int W, double* px, double* py) {
    *px = 1.0 - (2.0 * (double)c + 1.0) / (double)W;
    *py = 1.0 - (2.0 * (double)r + 1.0) / (double)H;
}

typedef struct {
    double z;
    int64_t id;
    double d2;
} pt_hit_t;

static int pt_hit_cmp(const void* pa, const void* pb) {
    const pt_hit_t* a = (const pt_hit_t*)pa;
    const pt_hit_t* b = (const pt_hit_t*)pb;
    if (a->z < b->z) return -1;
    if (a->z > b->z) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/*
 * points (P,3) FP64, clouds [first[n], first[n] + np[n]) for image n.
 * pix: optional list of npix linear pixel ids (n*H*W + r*W + c); with it the
 * outputs are (npix, K) rows, else (N,H,W,K).  amb (per output pixel): bit 0
 * = some point's distance is within PT_TAU of the radius, bit 1 = two of the
 * first min(K+1, hits) sorted hits have z within PT_TAU, bit 2 = a covering
 * point has abs(z) < PT_TAU.  Returns 0, or -1 on a bad range or no memory.
 */
int oracle_points_rasterize(const double* points, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                            int W, double radius, int K, const int64_t* pix, int64_t npix, int64_t* idx,
                            double* zbuf, double* dists, uint8_t* amb, int nthreads) {
    for (int n = 0; n < N; ++n)
        if (first[n] < 0 || np[n] < 0 || first[n] + np[n] > P) return -1;
    const int64_t total = pix ? npix : (int64_t)N * H * W;
    const double r2 = radius * radius;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t cap = 64;
        pt_hit_t* hits = (pt_hit_t*)malloc(sizeof(pt_hit_t) * cap);
        if (!hits) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < total; ++t) {
            if (!hits) continue;
            const int64_t lin = pix ? pix[t] : t;
            const int n = (int)(lin / ((int64_t)H * W));
            const int64_t rem = lin % ((int64_t)H * W);
            double px, py;
            pt_pixel_center(rem / W, rem % W, H, W, &px, &py);
            int64_t nh = 0;
            uint8_t a = 0;
            for (int64_t p = first[n]; p < first[n] + np[n]; ++p) {
                const double dx = points[3 * p] - px, dy = points[3 * p + 1] - py, z = points[3 * p + 2];
                const double d2 = dx * dx + dy * dy;
                const double d = sqrt(d2);
                if (fabs(d - radius) < PT_TAU) a |= 1;
                if (!(d2 < r2) || z < 0.0) continue;
                if (fabs(z) < PT_TAU) a |= 4;
                if (nh == cap) {
                    cap *= 2;
                    pt_hit_t* h2 = (pt_hit_t*)realloc(hits, sizeof(pt_hit_t) * cap);
                    if (!h2) {
#pragma omp atomic write
                        bad = 1;
                        break;
                    }
                    hits = h2;
                }
                hits[nh].z = z;
                hits[nh].id = p;
                hits[nh].d2 = d2;
                ++nh;
            }
            qsort(hits, (size_t)nh, sizeof(pt_hit_t), pt_hit_cmp);
            const int64_t lim = nh < K + 1 ? nh : K + 1;
            for (int64_t i = 1; i < lim; ++i)
                if (hits[i].z - hits[i - 1].z < PT_TAU) a |= 2;
            for (int k = 0; k < K; ++k) {
                const int64_t o = t * K + k;
                if (k < nh) {
                    idx[o] = hits[k].id;
                    zbuf[o] = hits[k].z;
                    dists[o] = hits[k].d2;
                } else {
                    idx[o] = -1;
                    zbuf[o] = -1.0;
                    dists[o] = -1.0;
                }
            }
            if (amb) amb[t] = a;
        }
        free(hits);
    }
    return bad ? -1 : 0;
}

/*
 * dL/dpoints (P,3) for the fixed choice idx: rows of pixels `pix` (npix
 * rows) or the full (N,H,W,K) grid when pix is NULL.  gz/gd may be NULL.
 */
int oracle_points_backward(const double* points, int64_t P, int N, int H, int W, int K, const int64_t* pix,
                           int64_t npix, const int64_t* idx, const double* gz, const double* gd, double* grad,
                           int nthreads) {
    const int64_t rows = pix ? npix : (int64_t)N * H * W;
    memset(grad, 0, sizeof(double) * 3 * (size_t)P);
    int nt = nthreads > 0 ? nthreads : 1;
    double* part = (double*)calloc((size_t)nt * 3 * (size_t)P, sizeof(double));
    if (!part) return -1;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* g = part + (size_t)tid * 3 * (size_t)P;
#pragma omp for schedule(static)
        for (int64_t t = 0; t < rows; ++t) {
            const int64_t lin = pix ? pix[t] : t;
            const int64_t rem = lin % ((int64_t)H * W);
            double px, py;
            pt_pixel_center(rem / W, rem % W, H, W, &px, &py);
            for (int k = 0; k < K; ++k) {
                const int64_t o = t * K + k;
                const int64_t p = idx[o];
                if (p < 0 || p >= P) continue;
                if (gz) g[3 * p + 2] += gz[o];
                if (gd) {
                    g[3 * p + 0] += 2.0 * gd[o] * (points[3 * p] - px);
                    g[3 * p + 1] += 2.0 * gd[o] * (points[3 * p + 1] - py);
                }
            }
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int64_t i = 0; i < 3 * P; ++i) grad[i] += part[(size_t)t * 3 * (size_t)P + i];
    free(part);
    return 0;
}
