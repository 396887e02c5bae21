/*
 * oracle_rast.c -- FP64 brute-force oracle for the batched mesh rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant generator with
 * the HIP library.
 *
 * What it computes (paper, Section 3.2 "Rasterizer"): for every pixel, the K
 * faces nearest along z among those that cover the pixel in the xy-plane or lie
 * within the blur radius of it, with the face id, the barycentric coordinates
 * of the pixel in the face, the interpolated z, and the signed xy distance from
 * the pixel to the face.  The paper reaches this set with tiles and per-pixel
 * priority queues; both are pure accelerations, so the oracle is the plain
 * definition: test every pixel against every face of its own mesh in FP64,
 * sort the hits by (z, face id), keep the first K.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - pixel (r, c) of an H x W image has its centre at
 *      x = 1 - (2c + 1) / W,  y = 1 - (2r + 1) / H   (+x left, +y up, row 0 top)
 *  - barycentrics are raw screen-space ones: w0 = cross(b-p, c-p) / E,
 *    w1 = cross(c-p, a-p) / E, w2 = cross(a-p, b-p) / E with
 *    E = cross(b-a, c-a) and cross(u, v) = u.x v.y - u.y v.x
 *  - z = w0 a.z + w1 b.z + w2 c.z
 *  - "inside" means all three w_i > 0 (strict)
 *  - d2 is the squared xy distance from the pixel centre to the nearest point
 *    of the triangle's boundary (its three edge segments); dists = -d2 inside,
 *    +d2 outside; blur_radius is in the same squared units
 *  - a face counts for a pixel iff (inside or d2 < blur_radius), z >= 0 and
 *    abs(E) >= 1e-8 (degenerate faces never count)
 *  - order: ascending z, then ascending packed face id
 *  - empty slots: face id -1 and -1 in zbuf, all three bary and dists
 *  - face ids are packed global ids (indices into the packed face array)
 *
 * Rasterizer options (bits of `opts`; the paper fixes none of them, these are
 * the readings):
 *  - ORC_CULL: a face whose doubled signed area E in the x-y NDC plane is
 *    positive never counts (with +x to the left, E < 0 is anticlockwise as
 *    the image is displayed, the usual front-facing order)
 *  - ORC_PERSPECTIVE: the barycentrics are perspective-corrected,
 *    w'_i = (w_i / z_i) / sum_j (w_j / z_j) with the vertex depths z_i; a face
 *    with a vertex at z <= 0 never counts, nor does a pair whose
 *    sum_j (w_j / z_j) is not positive
 *  - ORC_CLIP: the barycentrics (after the correction) are clipped,
 *    w''_i = max(w_i, 0) / sum_j max(w_j, 0)
 *  - z is interpolated with the final barycentrics, and the z >= 0 test and
 *    the order use it; "inside" and dists keep using the raw barycentrics
 *    and the geometry
 *
 * Ambiguity mask (decision margin tau = 1e-6 in linear NDC units): a pixel is
 * flagged when a rounding-level change of the inputs could change its face
 * selection; exact equality of the face ids is only claimed on unflagged
 * pixels (any valid answer is still checked there, see oracle_candidates).
 *    M1 blur == 0 and some face passes within tau of the pixel centre
 *    M2 blur > 0 and some face that does not contain the pixel has
 *       abs(sqrt(d2) - sqrt(blur)) < tau
 *    M3 the set of K faces is tied: the K-th and the (K+1)-th sorted hits
 *       differ in z by less than tau
 *    M4 some face that covers the pixel has abs(z) < tau
 *    M5 some face that would cover the pixel if it were not degenerate (or
 *       that does cover it) has abs(abs(E) - 1e-8) < 1e-3 * 1e-8
 *    M6 (per slot, gradients only) the two smallest edge distances of the
 *       slot's face differ by less than tau (in linear units)
 *    M7 (perspective correction) a face that passes the coverage test has a
 *       vertex depth within tau of 0, or sum_j (w_j / z_j) within tau of 0
 *    M8 only the order is tied: two neighbours among the first K sorted hits
 *       differ in z by less than tau (the set of K faces is still unique, the
 *       order inside each run of tied hits is not)
 * M1, M2, M4, M5 and M7 are also recorded per face by oracle_candidates,
 * which lists every face that counts or nearly counts for a pixel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TAU 1e-6
#define ORC_EPS_AREA 1e-8

#define AMB_M1 1
#define AMB_M2 2
#define AMB_M3 4
#define AMB_M4 8
#define AMB_M5 16
#define AMB_M7 64
#define AMB_M8 128

/* per-face classes of oracle_candidates */
#define CLS_COUNTS 0     /* counts, and no margin case applies to it */
#define CLS_BORDER_IN 1  /* counts, but within a margin of not counting */
#define CLS_BORDER_OUT 2 /* does not count, but within a margin of counting */

#define ORC_PERSPECTIVE 0x100
#define ORC_CLIP 0x200
#define ORC_CULL 0x400

typedef struct {
    double z;
    int64_t f;
    double w[3];
    double sd; /* signed squared distance */
    int cls;   /* CLS_* */
} hit_t;

static double cross2(double ux, double uy, double vx, double vy) { return ux * vy - uy * vx; }

static void pixel_center(int64_t r, int64_t c, int H, int W, double* px, double* py) {
    *px = 1.0 - (2.0 * (double)c + 1.0) / (double)W;
    *py = 1.0 - (2.0 * (double)r + 1.0) / (double)H;
}

/* Squared distance from p to segment s-t and the segment parameter u of the
 * closest point q = s + u (t - s), u clamped to [0, 1].  A zero-length segment
 * gives the distance to s. */
static double seg_d2(double px, double py, double sx, double sy, double tx, double ty, double* u_out) {
    double vx = tx - sx, vy = ty - sy;
    double l2 = vx * vx + vy * vy;
    double u = 0.0;
    if (l2 > 0.0) {
        u = ((px - sx) * vx + (py - sy) * vy) / l2;
        if (u < 0.0) u = 0.0;
        if (u > 1.0) u = 1.0;
    }
    double qx = sx + u * vx, qy = sy + u * vy;
    if (u_out) *u_out = u;
    return (px - qx) * (px - qx) + (py - qy) * (py - qy);
}

typedef struct {
    double E;
    double w[3];  /* raw screen-space barycentrics */
    double wp[3]; /* after the perspective correction (= w without it) */
    double wf[3]; /* final: after the correction and the clipping */
    double D;     /* sum_j w_j / z_j (perspective correction) */
    double M;     /* sum_j max(wp_j, 0) (clipping) */
    double zf;    /* depth interpolated with wf */
    int opts_ok;  /* the options admit the pair */
    double z;
    double d2;
    double de[3]; /* squared distance to each edge e0=(a,b), e1=(b,c), e2=(c,a) */
    double u[3];
    int inside;
    int argmin; /* lowest edge index among the minimal ones */
} eval_t;

/* The options' barycentrics and depth from the raw ones (see the header). */
static void apply_options(int opts, const double* a, const double* b, const double* c, eval_t* ev) {
    const double Z[3] = {a[2], b[2], c[2]};
    ev->opts_ok = 1;
    ev->D = 1.0;
    ev->M = 1.0;
    for (int i = 0; i < 3; ++i) ev->wp[i] = ev->w[i];
    if (opts & ORC_PERSPECTIVE) {
        if (!(Z[0] > 0.0 && Z[1] > 0.0 && Z[2] > 0.0)) {
            ev->opts_ok = 0;
        } else {
            double u[3];
            for (int i = 0; i < 3; ++i) u[i] = ev->w[i] / Z[i];
            ev->D = u[0] + u[1] + u[2];
            if (!(ev->D > 0.0)) ev->opts_ok = 0;
            else
                for (int i = 0; i < 3; ++i) ev->wp[i] = u[i] / ev->D;
        }
    }
    for (int i = 0; i < 3; ++i) ev->wf[i] = ev->wp[i];
    if ((opts & ORC_CLIP) && ev->opts_ok) {
        double m[3];
        for (int i = 0; i < 3; ++i) m[i] = ev->wp[i] > 0.0 ? ev->wp[i] : 0.0;
        ev->M = m[0] + m[1] + m[2];
        if (!(ev->M > 0.0)) ev->opts_ok = 0;
        else
            for (int i = 0; i < 3; ++i) ev->wf[i] = m[i] / ev->M;
    }
    ev->zf = ev->wf[0] * Z[0] + ev->wf[1] * Z[1] + ev->wf[2] * Z[2];
}

/* Evaluate face (a, b, c) at pixel p under the options.  Returns 0 if the
 * face is degenerate (abs(E) < 1e-8); its values are still filled in when
 * E != 0, for the margin test M5. */
static int eval_face(const double* a, const double* b, const double* c, double px, double py, int opts,
                          eval_t* ev) {
    double E = cross2(b[0] - a[0], b[1] - a[1], c[0] - a[0], c[1] - a[1]);
    ev->E = E;
    if (E == 0.0) return 0;
    double e0 = cross2(b[0] - px, b[1] - py, c[0] - px, c[1] - py);
    double e1 = cross2(c[0] - px, c[1] - py, a[0] - px, a[1] - py);
    double e2 = cross2(a[0] - px, a[1] - py, b[0] - px, b[1] - py);
    ev->w[0] = e0 / E;
    ev->w[1] = e1 / E;
    ev->w[2] = e2 / E;
    ev->z = ev->w[0] * a[2] + ev->w[1] * b[2] + ev->w[2] * c[2];
    ev->inside = (ev->w[0] > 0.0) && (ev->w[1] > 0.0) && (ev->w[2] > 0.0);
    ev->de[0] = seg_d2(px, py, a[0], a[1], b[0], b[1], &ev->u[0]);
    ev->de[1] = seg_d2(px, py, b[0], b[1], c[0], c[1], &ev->u[1]);
    ev->de[2] = seg_d2(px, py, c[0], c[1], a[0], a[1], &ev->u[2]);
    int am = 0;
    if (ev->de[1] < ev->de[am]) am = 1;
    if (ev->de[2] < ev->de[am]) am = 2;
    ev->argmin = am;
    ev->d2 = ev->de[am];
    apply_options(opts, a, b, c, ev);
    return fabs(E) >= ORC_EPS_AREA;
}

static int hit_cmp(const void* pa, const void* pb) {
    const hit_t* a = (const hit_t*)pa;
    const hit_t* b = (const hit_t*)pb;
    if (a->z < b->z) return -1;
    if (a->z > b->z) return 1;
    if (a->f < b->f) return -1;
    if (a->f > b->f) return 1;
    return 0;
}

static void load_vert(const double* verts, int64_t vi, double* out) {
    out[0] = verts[3 * vi + 0];
    out[1] = verts[3 * vi + 1];
    out[2] = verts[3 * vi + 2];
}

/* Every face of mesh n tested at pixel centre p: appends to *hits (grown
 * as needed) the faces that count, and with want_border also those that do
 * not count but lie within a margin of counting (class CLS_BORDER_OUT);
 * ORs the per-face margin bits M1, M2, M4, M5, M7 into *am.  Returns the
 * number of records, or -1 when memory runs out. */
static int64_t pixel_hits(const double* verts, const int64_t* faces, const int64_t* first, const int64_t* nfaces,
                          int64_t n, double px, double py, double blur, int opts, int want_border, hit_t** hits,
                          int64_t* cap, uint8_t* am) {
    const double sqrt_blur = sqrt(blur);
    int64_t nh = 0;
    for (int64_t f = first[n]; f < first[n] + nfaces[n]; ++f) {
        double a[3], b[3], cc[3];
        load_vert(verts, faces[3 * f + 0], a);
        load_vert(verts, faces[3 * f + 1], b);
        load_vert(verts, faces[3 * f + 2], cc);
        eval_t ev;
        const int nondegen = eval_face(a, b, cc, px, py, opts, &ev);
        if (ev.E == 0.0) continue;
        if ((opts & ORC_CULL) && ev.E > 0.0) continue;
        /* the four conditions of counting, each with the margin bit that
         * makes its outcome uncertain */
        const double dist = sqrt(ev.d2);
        const int covers = ev.inside || (ev.d2 < blur);
        uint8_t b_cov = 0;
        if (blur == 0.0) {
            if (dist < ORC_TAU) b_cov = AMB_M1;
        } else if (!ev.inside && fabs(dist - sqrt_blur) < ORC_TAU) {
            b_cov = AMB_M2;
        }
        const uint8_t b_nd = fabs(fabs(ev.E) - ORC_EPS_AREA) < 1e-3 * ORC_EPS_AREA ? AMB_M5 : 0;
        uint8_t b_opt = 0;
        if ((opts & ORC_PERSPECTIVE) &&
            (fabs(a[2]) < ORC_TAU || fabs(b[2]) < ORC_TAU || fabs(cc[2]) < ORC_TAU || fabs(ev.D) < ORC_TAU))
            b_opt = AMB_M7;
        const int z_ok = ev.zf >= 0.0;
        const uint8_t b_z = fabs(ev.zf) < ORC_TAU ? AMB_M4 : 0;
        const int counts = nondegen && covers && ev.opts_ok && z_ok;
        /* could it count under a rounding-level change?  Each condition holds
         * or is on its margin. */
        const int could = (nondegen || b_nd) && (covers || b_cov) && (ev.opts_ok || b_opt) && (z_ok || b_z);
        if (!could) continue;
        const uint8_t fb = b_cov | b_nd | b_opt | b_z;
        *am |= fb;
        if (!counts && !want_border) continue;
        if (nh == *cap) {
            int64_t ncap = *cap * 2;
            hit_t* nhp = (hit_t*)realloc(*hits, sizeof(hit_t) * (size_t)ncap);
            if (!nhp) return -1;
            *hits = nhp;
            *cap = ncap;
        }
        hit_t* h = &(*hits)[nh++];
        h->z = ev.zf;
        h->f = f;
        h->w[0] = ev.wf[0];
        h->w[1] = ev.wf[1];
        h->w[2] = ev.wf[2];
        h->sd = ev.inside ? -ev.d2 : ev.d2;
        h->cls = counts ? (fb ? CLS_BORDER_IN : CLS_COUNTS) : CLS_BORDER_OUT;
    }
    return nh;
}

/* Order-tie bits of a pixel from its sorted hits (faces that count only):
 * M3 when the K-th and (K+1)-th differ in z by less than tau, M8 when two
 * neighbours among the first K do. */
static uint8_t tie_bits(const hit_t* hits, int64_t nh, int K) {
    uint8_t am = 0;
    if (nh > K && fabs(hits[K].z - hits[K - 1].z) < ORC_TAU) am |= AMB_M3;
    int64_t lim = nh < (int64_t)K ? nh : (int64_t)K;
    for (int64_t j = 0; j + 1 < lim; ++j)
        if (fabs(hits[j + 1].z - hits[j].z) < ORC_TAU) am |= AMB_M8;
    return am;
}

/*
 * Forward over a list of pixels.
 *   verts (V,3) f64, faces (F,3) i64 global vertex ids, first/nfaces (N) i64
 *   pix: linear pixel ids n*H*W + r*W + c (npix of them); NULL = every pixel
 *   outputs per listed pixel i (row-major like the pixel list):
 *     p2f (npix,K) i64, zbuf (npix,K), bary (npix,K,3), dists (npix,K) f64,
 *     amb (npix) u8 bit mask of M1..M5, M7, M8 (may be NULL),
 *     nhits (npix) i64 (may be NULL)
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_rasterize(const double* verts, int64_t V, const int64_t* faces, int64_t F,
                     const int64_t* first, const int64_t* nfaces, int N, int H, int W,
                     double blur, int K, const int64_t* pix, int64_t npix,
                     int64_t* p2f, double* zbuf, double* bary, double* dists,
                     uint8_t* amb, int64_t* nhits, int opts, int nthreads) {
    if (N < 0 || H <= 0 || W <= 0 || K <= 0 || blur < 0.0) return -1;
    int64_t total = (int64_t)N * H * W;
    if (pix == NULL) npix = total;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t cap = 256;
        hit_t* hits = (hit_t*)malloc(sizeof(hit_t) * cap);
        if (!hits) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < npix; ++i) {
            if (!hits) continue;
            int64_t lin = pix ? pix[i] : i;
            int64_t n = lin / ((int64_t)H * W);
            int64_t rem = lin % ((int64_t)H * W);
            int64_t r = rem / W, c = rem % W;
            double px, py;
            pixel_center(r, c, H, W, &px, &py);
            uint8_t am = 0;
            if (n < 0 || n >= N) {
                bad = 1;
                continue;
            }
            int64_t nh = pixel_hits(verts, faces, first, nfaces, n, px, py, blur, opts, 0, &hits, &cap, &am);
            if (nh < 0) {
                bad = 1;
                continue;
            }
            qsort(hits, (size_t)nh, sizeof(hit_t), hit_cmp);
            am |= tie_bits(hits, nh, K);
            for (int k = 0; k < K; ++k) {
                int64_t o = i * K + k;
                if (k < nh) {
                    p2f[o] = hits[k].f;
                    zbuf[o] = hits[k].z;
                    bary[3 * o + 0] = hits[k].w[0];
                    bary[3 * o + 1] = hits[k].w[1];
                    bary[3 * o + 2] = hits[k].w[2];
                    dists[o] = hits[k].sd;
                } else {
                    p2f[o] = -1;
                    zbuf[o] = -1.0;
                    bary[3 * o + 0] = bary[3 * o + 1] = bary[3 * o + 2] = -1.0;
                    dists[o] = -1.0;
                }
            }
            if (amb) amb[i] = am;
            if (nhits) nhits[i] = nh;
        }
        free(hits);
    }
    (void)V;
    (void)F;
    return bad ? -1 : 0;
}

/*
 * Every face that counts for a listed pixel, or lies within a margin of
 * counting (M1, M2, M4, M5, M7 of that face), sorted by (z, face id): the
 * material to decide whether some other answer than oracle_rasterize's is
 * also correct for a flagged pixel.  Per pixel i, up to cap records:
 *   cf (npix,cap) i64 face id (-1 past the end), cz (npix,cap) z,
 *   cw (npix,cap,3) barycentrics, cd (npix,cap) signed squared distance,
 *   ccls (npix,cap) u8 class (CLS_COUNTS, CLS_BORDER_IN, CLS_BORDER_OUT),
 *   ncand (npix) i64 the number of such faces (may exceed cap: then only
 *   the first cap are listed).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_candidates(const double* verts, const int64_t* faces, const int64_t* first, const int64_t* nfaces,
                      int N, int H, int W, double blur, const int64_t* pix, int64_t npix, int cap_out,
                      int64_t* cf, double* cz, double* cw, double* cd, uint8_t* ccls, int64_t* ncand, int opts,
                      int nthreads) {
    if (N < 0 || H <= 0 || W <= 0 || cap_out <= 0 || blur < 0.0 || pix == NULL) return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t cap = 256;
        hit_t* hits = (hit_t*)malloc(sizeof(hit_t) * cap);
        if (!hits) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < npix; ++i) {
            if (!hits) continue;
            int64_t lin = pix[i];
            int64_t n = lin / ((int64_t)H * W);
            int64_t rem = lin % ((int64_t)H * W);
            double px, py;
            pixel_center(rem / W, rem % W, H, W, &px, &py);
            if (n < 0 || n >= N) {
                bad = 1;
                continue;
            }
            uint8_t am = 0;
            int64_t nh = pixel_hits(verts, faces, first, nfaces, n, px, py, blur, opts, 1, &hits, &cap, &am);
            if (nh < 0) {
                bad = 1;
                continue;
            }
            qsort(hits, (size_t)nh, sizeof(hit_t), hit_cmp);
            for (int k = 0; k < cap_out; ++k) {
                int64_t o = i * cap_out + k;
                if (k < nh) {
                    cf[o] = hits[k].f;
                    cz[o] = hits[k].z;
                    cw[3 * o + 0] = hits[k].w[0];
                    cw[3 * o + 1] = hits[k].w[1];
                    cw[3 * o + 2] = hits[k].w[2];
                    cd[o] = hits[k].sd;
                    ccls[o] = (uint8_t)hits[k].cls;
                } else {
                    cf[o] = -1;
                    cz[o] = cd[o] = -1.0;
                    cw[3 * o + 0] = cw[3 * o + 1] = cw[3 * o + 2] = -1.0;
                    ccls[o] = 255;
                }
            }
            ncand[i] = nh;
        }
        free(hits);
    }
    return bad ? -1 : 0;
}

/*
 * Fragment values for a FIXED selection: for every slot (n,r,c,k) with
 * p2f >= 0, recompute bary, z and signed distance of that face at that pixel
 * in FP64; empty slots get -1.  This is the forward map with the face choice
 * frozen, used for finite-difference checks of the backward.
 * Also writes tie (per slot, may be NULL): 1 where the two smallest edge
 * distances differ by less than tau in linear units (M6).
 * With pix (npix linear pixel ids) the slots are the rows of those pixels.
 */
int oracle_fragments_fixed(const double* verts, const int64_t* faces, int N, int H, int W, int K,
                           const int64_t* pix, int64_t npix, const int64_t* p2f, double* zbuf, double* bary,
                           double* dists, uint8_t* tie, int opts, int nthreads) {
    int64_t S = pix ? npix * K : (int64_t)N * H * W * K;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t s = 0; s < S; ++s) {
        int64_t f = p2f[s];
        if (tie) tie[s] = 0;
        if (f < 0) {
            zbuf[s] = -1.0;
            bary[3 * s] = bary[3 * s + 1] = bary[3 * s + 2] = -1.0;
            dists[s] = -1.0;
            continue;
        }
        int64_t lin = pix ? pix[s / K] : s / K;
        int64_t rem = lin % ((int64_t)H * W);
        double px, py;
        pixel_center(rem / W, rem % W, H, W, &px, &py);
        double a[3], b[3], c[3];
        load_vert(verts, faces[3 * f + 0], a);
        load_vert(verts, faces[3 * f + 1], b);
        load_vert(verts, faces[3 * f + 2], c);
        eval_t ev;
        if (!eval_face(a, b, c, px, py, opts, &ev) || !ev.opts_ok) {
            /* a degenerate face (or one the options exclude) can only appear
             * here if the caller's selection came from perturbed inputs;
             * report NaN so it cannot go unnoticed */
            zbuf[s] = NAN;
            bary[3 * s] = bary[3 * s + 1] = bary[3 * s + 2] = NAN;
            dists[s] = NAN;
            continue;
        }
        zbuf[s] = ev.zf;
        bary[3 * s + 0] = ev.wf[0];
        bary[3 * s + 1] = ev.wf[1];
        bary[3 * s + 2] = ev.wf[2];
        dists[s] = ev.inside ? -ev.d2 : ev.d2;
        if (tie) {
            double d[3] = {sqrt(ev.de[0]), sqrt(ev.de[1]), sqrt(ev.de[2])};
            double m1 = d[ev.argmin];
            double m2 = INFINITY;
            for (int e = 0; e < 3; ++e)
                if (e != ev.argmin && d[e] < m2) m2 = d[e];
            tie[s] = (m2 - m1) < ORC_TAU;
        }
    }
    return 0;
}

/*
 * Analytic backward (paper, Section 3.2: the renderer gives gradients with
 * respect to its inputs, and the backward reuses the stored face choice).
 *
 * Loss L = sum_slots gz*z + sum_i gb_i*w_i + gd*dists over slots with
 * p2f >= 0; returns dL/dverts (V,3), zeroed first.  gz/gb/gd may be NULL (=0).
 *
 * Derivatives, with p the pixel centre fixed:
 *   d cross(u,v)/du = (v.y, -v.x),  d cross(u,v)/dv = (-u.y, u.x)
 *   e0 = cross(b-p, c-p), e1 = cross(c-p, a-p), e2 = cross(a-p, b-p), E = e0+e1+e2
 *   dw_i/dv = (de_i/dv - w_i dE/dv) / E  for the xy of each vertex v
 *   z = sum_i w_i z_i:  dz/dv_xy = sum_i z_i dw_i/dv_xy,  dz/dz_i = w_i
 *   dists = s * d2 with s = -1 inside, +1 outside (piecewise constant);
 *   on the nearest edge (s0, t) with closest point q = s0 + u (t - s0):
 *   d d2/d s0 = -2 (1-u) (p-q),  d d2/d t = -2 u (p-q)   (also at clamped u)
 * With the options the outputs are the final barycentrics wf and
 * zf = sum_i wf_i z_i; with G_i = dL/dwf_i = gb_i + gz z_i (and dL/dz_i += gz wf_i):
 *   clipping wf_i = m_i / M, m_i = max(wp_i, 0):
 *     dL/dwp_j = (G_j - sum_i G_i wf_i) / M where wp_j > 0, else 0
 *   correction wp_i = u_i / D, u_i = w_i / z_i, D = sum_j u_j:
 *     dL/du_j = (Gp_j - sum_i Gp_i wp_i) / D,
 *     dL/dw_j = dL/du_j / z_j,  dL/dz_j += -dL/du_j w_j / z_j^2
 *   and dL/dw (raw) enters the xy chain above.
 */
int oracle_backward(const double* verts, int64_t V, const int64_t* faces, int N, int H, int W, int K,
                    const int64_t* pix, int64_t npix,
                    const int64_t* p2f, const double* gz, const double* gb, const double* gd,
                    double* grad_verts, int opts, int nthreads) {
    int nt = nthreads > 0 ? nthreads : 1;
    /* pix == NULL: slots cover every pixel in order, S = N*H*W*K; otherwise
     * slot s belongs to linear pixel pix[s / K] and S = npix*K */
    int64_t S = pix ? npix * K : (int64_t)N * H * W * K;
    double* part = (double*)calloc((size_t)nt * (size_t)V * 3, sizeof(double));
    if (!part && V > 0) return -1;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* g = part + (size_t)tid * (size_t)V * 3;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < S; ++s) {
            int64_t f = p2f[s];
            if (f < 0) continue;
            double gzs = gz ? gz[s] : 0.0;
            double gb0 = gb ? gb[3 * s + 0] : 0.0;
            double gb1 = gb ? gb[3 * s + 1] : 0.0;
            double gb2 = gb ? gb[3 * s + 2] : 0.0;
            double gds = gd ? gd[s] : 0.0;
            int64_t lin = pix ? pix[s / K] : s / K;
            int64_t rem = lin % ((int64_t)H * W);
            double px, py;
            pixel_center(rem / W, rem % W, H, W, &px, &py);
            int64_t vi[3] = {faces[3 * f + 0], faces[3 * f + 1], faces[3 * f + 2]};
            double P[3][3];
            for (int j = 0; j < 3; ++j) load_vert(verts, vi[j], P[j]);
            eval_t ev;
            if (!eval_face(P[0], P[1], P[2], px, py, opts, &ev) || !ev.opts_ok) continue;
            double E = ev.E;
            /* relative positions r_j = P_j - p */
            double rx[3], ry[3];
            for (int j = 0; j < 3; ++j) {
                rx[j] = P[j][0] - px;
                ry[j] = P[j][1] - py;
            }
            /* de_i/dP_j (xy), e_i = cross(r_{i+1}, r_{i+2}) (indices mod 3) */
            double de[3][3][2];
            memset(de, 0, sizeof(de));
            for (int i = 0; i < 3; ++i) {
                int u = (i + 1) % 3, v = (i + 2) % 3;
                /* d cross(r_u, r_v)/d r_u = (r_v.y, -r_v.x); d/d r_v = (-r_u.y, r_u.x) */
                de[i][u][0] = ry[v];
                de[i][u][1] = -rx[v];
                de[i][v][0] = -ry[u];
                de[i][v][1] = rx[u];
            }
            double G[3];
            double Z[3] = {P[0][2], P[1][2], P[2][2]};
            G[0] = gb0 + gzs * Z[0];
            G[1] = gb1 + gzs * Z[1];
            G[2] = gb2 + gzs * Z[2];
            for (int j = 0; j < 3; ++j) g[3 * vi[j] + 2] += gzs * ev.wf[j];
            if (opts & ORC_CLIP) {
                double S = G[0] * ev.wf[0] + G[1] * ev.wf[1] + G[2] * ev.wf[2];
                for (int i = 0; i < 3; ++i) G[i] = ev.wp[i] > 0.0 ? (G[i] - S) / ev.M : 0.0;
            }
            if (opts & ORC_PERSPECTIVE) {
                double S = G[0] * ev.wp[0] + G[1] * ev.wp[1] + G[2] * ev.wp[2];
                for (int i = 0; i < 3; ++i) {
                    double gu = (G[i] - S) / ev.D;
                    G[i] = gu / Z[i];
                    g[3 * vi[i] + 2] += -gu * ev.w[i] / (Z[i] * Z[i]);
                }
            }
            for (int j = 0; j < 3; ++j) {
                for (int x = 0; x < 2; ++x) {
                    double dE = de[0][j][x] + de[1][j][x] + de[2][j][x];
                    double acc = 0.0;
                    for (int i = 0; i < 3; ++i) {
                        double dw = (de[i][j][x] - ev.w[i] * dE) / E;
                        acc += G[i] * dw;
                    }
                    g[3 * vi[j] + x] += acc;
                }
            }
            if (gds != 0.0) {
                double sgn = ev.inside ? -1.0 : 1.0;
                int e = ev.argmin;
                int js = e, jt = (e + 1) % 3; /* e0=(a,b), e1=(b,c), e2=(c,a) */
                double u = ev.u[e];
                double qx = P[js][0] + u * (P[jt][0] - P[js][0]);
                double qy = P[js][1] + u * (P[jt][1] - P[js][1]);
                double dx = px - qx, dy = py - qy;
                g[3 * vi[js] + 0] += sgn * gds * (-2.0 * (1.0 - u) * dx);
                g[3 * vi[js] + 1] += sgn * gds * (-2.0 * (1.0 - u) * dy);
                g[3 * vi[jt] + 0] += sgn * gds * (-2.0 * u * dx);
                g[3 * vi[jt] + 1] += sgn * gds * (-2.0 * u * dy);
            }
        }
    }
    for (int64_t q = 0; q < V * 3; ++q) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * (size_t)V * 3 + (size_t)q];
        grad_verts[q] = s;
    }
    free(part);
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
