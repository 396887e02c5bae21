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
 * selection; parity of the face ids is only claimed on unflagged pixels.
 *    M1 blur == 0 and some face passes within tau of the pixel centre
 *    M2 blur > 0 and some face that does not contain the pixel has
 *       abs(sqrt(d2) - sqrt(blur)) < tau
 *    M3 two neighbours among the first min(K+1, hits) sorted hits differ in z
 *       by less than tau
 *    M4 some face that covers the pixel has abs(z) < tau
 *    M5 some face has abs(abs(E) - 1e-8) < 1e-3 * 1e-8
 *    M6 (per slot, gradients only) the two smallest edge distances of the
 *       slot's face differ by less than tau (in linear units)
 *    M7 (perspective correction) a face that passes the coverage test has a
 *       vertex depth within tau of 0, or sum_j (w_j / z_j) within tau of 0
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

#define ORC_PERSPECTIVE 0x100
#define ORC_CLIP 0x200
#define ORC_CULL 0x400

typedef struct {
    double z;
    int64_t f;
    double w[3];
    double sd; /* signed squared distance */
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
 * face is degenerate. */
static int eval_face(const double* a, const double* b, const double* c, double px, double py, int opts,
                          eval_t* ev) {
    double E = cross2(b[0] - a[0], b[1] - a[1], c[0] - a[0], c[1] - a[1]);
    ev->E = E;
    if (fabs(E) < ORC_EPS_AREA) return 0;
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
    return 1;
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

/*
 * Forward over a list of pixels.
 *   verts (V,3) f64, faces (F,3) i64 global vertex ids, first/nfaces (N) i64
 *   pix: linear pixel ids n*H*W + r*W + c (npix of them); NULL = every pixel
 *   outputs per listed pixel i (row-major like the pixel list):
 *     p2f (npix,K) i64, zbuf (npix,K), bary (npix,K,3), dists (npix,K) f64,
 *     amb (npix) u8 bit mask of M1..M5 (may be NULL), nhits (npix) i64 (may be NULL)
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
    double sqrt_blur = sqrt(blur);
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
            int64_t nh = 0;
            uint8_t am = 0;
            if (n < 0 || n >= N) {
                bad = 1;
                continue;
            }
            for (int64_t f = first[n]; f < first[n] + nfaces[n]; ++f) {
                double a[3], b[3], cc[3];
                load_vert(verts, faces[3 * f + 0], a);
                load_vert(verts, faces[3 * f + 1], b);
                load_vert(verts, faces[3 * f + 2], cc);
                eval_t ev;
                int ok = eval_face(a, b, cc, px, py, opts, &ev);
                if (fabs(fabs(ev.E) - ORC_EPS_AREA) < 1e-3 * ORC_EPS_AREA) am |= AMB_M5;
                if (!ok) continue;
                if ((opts & ORC_CULL) && ev.E > 0.0) continue;
                double dist = sqrt(ev.d2);
                if (blur == 0.0) {
                    if (dist < ORC_TAU) am |= AMB_M1;
                } else if (!ev.inside && fabs(dist - sqrt_blur) < ORC_TAU) {
                    am |= AMB_M2;
                }
                int covers = ev.inside || (ev.d2 < blur);
                if (!covers) continue;
                if (opts & ORC_PERSPECTIVE) {
                    if (fabs(a[2]) < ORC_TAU || fabs(b[2]) < ORC_TAU || fabs(cc[2]) < ORC_TAU ||
                        fabs(ev.D) < ORC_TAU)
                        am |= AMB_M7;
                }
                if (!ev.opts_ok) continue;
                if (fabs(ev.zf) < ORC_TAU) am |= AMB_M4;
                if (ev.zf < 0.0) continue;
                if (nh == cap) {
                    cap *= 2;
                    hit_t* nhp = (hit_t*)realloc(hits, sizeof(hit_t) * cap);
                    if (!nhp) {
                        bad = 1;
                        break;
                    }
                    hits = nhp;
                }
                hit_t* h = &hits[nh++];
                h->z = ev.zf;
                h->f = f;
                h->w[0] = ev.wf[0];
                h->w[1] = ev.wf[1];
                h->w[2] = ev.wf[2];
                h->sd = ev.inside ? -ev.d2 : ev.d2;
            }
            qsort(hits, (size_t)nh, sizeof(hit_t), hit_cmp);
            int64_t lim = nh < (int64_t)K + 1 ? nh : (int64_t)K + 1;
            for (int64_t j = 0; j + 1 < lim; ++j)
                if (fabs(hits[j + 1].z - hits[j].z) < ORC_TAU) am |= AMB_M3;
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
