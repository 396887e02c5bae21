// kernels_bwd.hip -- backward of the rasterizer for gfx950.
//
// The forward stores only the face ids (paper, Section 3.2: the cached
// Fragment data avoid recomputing face-pixel intersections); the backward
// recomputes barycentrics, z and the nearest edge of every filled slot and
// sums the chain rule into the nine vertex coordinates of its face.  Two
// forms.  The binned form (the forward's bins): one workgroup per bin, the
// bin's faces in LDS, exact fixed-point sums per face (described with its
// kernels below).  The per-face form (no bins): the thread that owns face f
// scans the pixels of f's blur-grown bounding box (the only pixels whose
// slots the forward can fill with f), finds the slot holding f in each and
// sums in registers -- no atomics per slot; a workgroup then merges its 256
// faces' contributions per vertex in an LDS hash table and issues one float
// atomic per (vertex, coordinate).  Faces whose box exceeds kBigArea pixels
// are handed to a second kernel in which a whole workgroup scans one face's
// box.
//
// Derivatives (pixel p fixed, R_j = v_j - p, cross(u,v) = u.x v.y - u.y v.x):
//   e0 = cross(R1,R2), e1 = cross(R2,R0), e2 = cross(R0,R1), E = e0+e1+e2,
//   w_i = e_i / E.  With G_i = gbary_i + gzbuf * z_i and Gw = sum_i G_i w_i,
//   dL/dv_j(xy) = sum_i (G_i - Gw)/E * de_i/dv_j   (uses dE/dv = sum_i de_i/dv)
//   dL/dz_j     = gzbuf * w_j
//   dists = s d2 (s = -1 inside, +1 outside); on the nearest edge (s0, t) with
//   nearest point Q = R_s0 + u (R_t - R_s0) (relative to p):
//   d d2/d s0 = 2 (1-u) Q,  d d2/d t = 2 u Q.
#include "../../include/rast.h"
#include "device.hpp"
#include "launch.hpp"

namespace rast {

constexpr int kBwdBlock = 256;
constexpr int kHash = 1024;     // LDS hash entries per workgroup (>= 3 * kBwdBlock)
constexpr int kBigArea = 256;   // faces with larger pixel boxes go to the cooperative kernel

struct BwdArgs {
    const float* verts;
    const int32_t* faces;
    const int64_t* first;
    const int64_t* nf;
    const int32_t* p2f;
    const float* gz;
    const float* gb;
    const float* gd;
    float* grad;
    int* hdr;
    int* big;      // list of faces with large boxes
    int64_t V, F;
    int N, H, W, K;
    float rb;      // sqrt(blur_radius)
    int opts;      // rasterizer options (kOpt*)
    // binned form
    const FaceRec* recs;
    const int* counts;
    const int* lists;
    float* partial;    // (F, 4, 9): a face's nine coordinate sums in the i-th bin of its range
    unsigned char* pmask;  // (F, 4): partial row written by this call (the binned form; shares big's memory)
    int bs, nby, nbx, M;
    int reuse;         // records and bins come from the forward: check its signature first
    BinSig sig;        // the signature this call expects
};

// False (and the status flagged) when a backward that reuses the forward's
// bins finds another call's signature in the workspace.  Every thread of a
// workgroup reads the same words, so the answer is uniform.
__device__ __forceinline__ bool bins_usable(const BwdArgs& a) {
    if (!a.reuse) return true;
    bool same = true;
#pragma unroll
    for (int i = 0; i < kSigWords; ++i) same = same && (a.hdr[kHdrSig + i] == a.sig.w[i]);
    if (!same && threadIdx.x == 0) atomicOr(&a.hdr[kHdrStatus], kStatReuse);
    return same;
}

struct FaceGrad {
    float gx[3], gy[3], gzv[3];
};

// Upstream gradients of slot s (zero for an absent array).  They and the
// slots' face ids are read once, so the binned pass loads them non-temporally
// (the "nt" hint), leaving L2 to the face records that neighbouring bins share.
struct SlotUp {
    float gz, gb0, gb1, gb2, gd;
};
__device__ __forceinline__ SlotUp load_up(const BwdArgs& a, int64_t s) {
    SlotUp u;
    u.gz = a.gz ? __builtin_nontemporal_load(a.gz + s) : 0.0f;
    u.gb0 = u.gb1 = u.gb2 = 0.0f;
    if (a.gb) {
        u.gb0 = __builtin_nontemporal_load(a.gb + 3 * s + 0);
        u.gb1 = __builtin_nontemporal_load(a.gb + 3 * s + 1);
        u.gb2 = __builtin_nontemporal_load(a.gb + 3 * s + 2);
    }
    u.gd = a.gd ? __builtin_nontemporal_load(a.gd + s) : 0.0f;
    return u;
}

// Adds the contribution of a slot of face R at pixel p, with upstream gradients up, to g.
// kOpts = false compiles out the options' barycentrics (for calls without them).
template <class Rec, bool kOpts = true>
__device__ __forceinline__ void slot_grad_up(const BwdArgs& a, const Rec& R, const float (&vz)[3], const Pix& p,
                                             const SlotUp& up, FaceGrad& g) {
    Eval ev;
    eval_full(R, p, ev);
    const float gzs = up.gz, gb0 = up.gb0, gb1 = up.gb1, gb2 = up.gb2, gds = up.gd;
    // dL/dw for the output barycentrics; z = sum_i w_i z_i adds gz z_i
    float G0 = gb0 + gzs * vz[0];
    float G1 = gb1 + gzs * vz[1];
    float G2 = gb2 + gzs * vz[2];
    if (kOpts && (a.opts & (kOptPersp | kOptClip))) {
        // the outputs are the options' barycentrics: carry dL/dw back through
        // the clipping and the correction to the raw ones (and to the depths)
        const float w[3] = {ev.w0, ev.w1, ev.w2};
        float wp[3] = {w[0], w[1], w[2]}, D = 1.0f;
        if (a.opts & kOptPersp) {
            const float u0 = w[0] / vz[0], u1 = w[1] / vz[1], u2 = w[2] / vz[2];
            D = u0 + u1 + u2;
            wp[0] = u0 / D;
            wp[1] = u1 / D;
            wp[2] = u2 / D;
        }
        float wf[3] = {wp[0], wp[1], wp[2]}, M = 1.0f;
        if (a.opts & kOptClip) {
            const float m0 = fmaxf(wp[0], 0.0f), m1 = fmaxf(wp[1], 0.0f), m2 = fmaxf(wp[2], 0.0f);
            M = m0 + m1 + m2;
            wf[0] = m0 / M;
            wf[1] = m1 / M;
            wf[2] = m2 / M;
        }
        g.gzv[0] += gzs * wf[0];
        g.gzv[1] += gzs * wf[1];
        g.gzv[2] += gzs * wf[2];
        if (a.opts & kOptClip) {
            const float S = G0 * wf[0] + G1 * wf[1] + G2 * wf[2];
            G0 = wp[0] > 0.0f ? (G0 - S) / M : 0.0f;
            G1 = wp[1] > 0.0f ? (G1 - S) / M : 0.0f;
            G2 = wp[2] > 0.0f ? (G2 - S) / M : 0.0f;
        }
        if (a.opts & kOptPersp) {
            const float S = G0 * wp[0] + G1 * wp[1] + G2 * wp[2];
            const float q0 = (G0 - S) / D, q1 = (G1 - S) / D, q2 = (G2 - S) / D;
            G0 = q0 / vz[0];
            G1 = q1 / vz[1];
            G2 = q2 / vz[2];
            g.gzv[0] -= q0 * w[0] / (vz[0] * vz[0]);
            g.gzv[1] -= q1 * w[1] / (vz[1] * vz[1]);
            g.gzv[2] -= q2 * w[2] / (vz[2] * vz[2]);
        }
    } else {
        g.gzv[0] += gzs * ev.w0;
        g.gzv[1] += gzs * ev.w1;
        g.gzv[2] += gzs * ev.w2;
    }
    float Gw = G0 * ev.w0 + G1 * ev.w1 + G2 * ev.w2;
    float invE = R.invE;
    float H0 = (G0 - Gw) * invE, H1 = (G1 - Gw) * invE, H2 = (G2 - Gw) * invE;
    // vertex positions relative to the pixel
    float Rx[3], Ry[3];
    Rx[0] = -ev.sx;
    Ry[0] = -ev.sy;
    Rx[1] = Rx[0] + (float)R.ab.x;
    Ry[1] = Ry[0] + (float)R.ab.y;
    Rx[2] = Rx[0] + (float)R.ac.x;
    Ry[2] = Ry[0] + (float)R.ac.y;
    // de0/dR1 = (R2.y, -R2.x), de0/dR2 = (-R1.y, R1.x)
    // de1/dR2 = (R0.y, -R0.x), de1/dR0 = (-R2.y, R2.x)
    // de2/dR0 = (R1.y, -R1.x), de2/dR1 = (-R0.y, R0.x)
    g.gx[0] += H1 * (-Ry[2]) + H2 * Ry[1];
    g.gy[0] += H1 * Rx[2] + H2 * (-Rx[1]);
    g.gx[1] += H0 * Ry[2] + H2 * (-Ry[0]);
    g.gy[1] += H0 * (-Rx[2]) + H2 * Rx[0];
    g.gx[2] += H0 * (-Ry[1]) + H1 * Ry[0];
    g.gy[2] += H0 * Rx[1] + H1 * (-Rx[0]);
    if (gds != 0.0f) {
        int e = ev.edge;
        int js = e, jt = e == 2 ? 0 : e + 1;
        float u = ev.u;
        float Rsx = js == 0 ? Rx[0] : (js == 1 ? Rx[1] : Rx[2]);
        float Rsy = js == 0 ? Ry[0] : (js == 1 ? Ry[1] : Ry[2]);
        float Rtx = jt == 0 ? Rx[0] : (jt == 1 ? Rx[1] : Rx[2]);
        float Rty = jt == 0 ? Ry[0] : (jt == 1 ? Ry[1] : Ry[2]);
        float Qx = Rsx + u * (Rtx - Rsx);
        float Qy = Rsy + u * (Rty - Rsy);
        float sg = ev.inside ? -gds : gds;
        float cs = 2.0f * (1.0f - u) * sg, ct = 2.0f * u * sg;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float k = (j == js) ? cs : ((j == jt) ? ct : 0.0f);
            g.gx[j] += k * Qx;
            g.gy[j] += k * Qy;
        }
    }
}

template <class Rec, bool kOpts = true>
__device__ __forceinline__ void slot_grad(const BwdArgs& a, const Rec& R, const float (&vz)[3], const Pix& p,
                                          int64_t s, FaceGrad& g) {
    slot_grad_up<Rec, kOpts>(a, R, vz, p, load_up(a, s), g);
}

// Scans the K slots of pixel (n, r, c) for face f and accumulates every match.
__device__ __forceinline__ void scan_pixel(const BwdArgs& a, const FaceRec& R, const float (&vz)[3], int f, int n,
                                           int r, int c, FaceGrad& g) {
    const int64_t pix = ((int64_t)n * a.H + r) * a.W + c;
    const int32_t* row = a.p2f + pix * a.K;
    int first_k = -1;
    bool more = false;
    if ((a.K & 3) == 0) {
        const int4* row4 = reinterpret_cast<const int4*>(row);
        for (int k = 0; k < a.K; k += 4) {
            int4 v = row4[k >> 2];
            int h = (int)(v.x == f) + (int)(v.y == f) + (int)(v.z == f) + (int)(v.w == f);
            if (h > 0) {
                int hit = v.x == f ? 0 : (v.y == f ? 1 : (v.z == f ? 2 : 3));
                more = more || first_k >= 0 || h > 1;
                if (first_k < 0) first_k = k + hit;
            }
        }
    } else {
        for (int k = 0; k < a.K; ++k) {
            if (row[k] == f) {
                more = more || first_k >= 0;
                if (first_k < 0) first_k = k;
            }
        }
    }
    if (first_k < 0) return;
    Pix p = make_pix(r, c, a.H, a.W);
    slot_grad(a, R, vz, p, pix * a.K + first_k, g);
    if (more) {
        // the same face in several slots of one pixel cannot come from the
        // forward, but every slot is still honoured
        for (int kk = first_k + 1; kk < a.K; ++kk)
            if (row[kk] == f) slot_grad(a, R, vz, p, pix * a.K + kk, g);
    }
}

// Face f's record (with the blur-grown box), its vertex ids and depths.
__device__ __forceinline__ bool load_face(const BwdArgs& a, int64_t f, FaceRec& R, int (&vi)[3], float (&vz)[3],
                                          int& n) {
    vi[0] = a.faces[3 * f];
    vi[1] = a.faces[3 * f + 1];
    vi[2] = a.faces[3 * f + 2];
    if (vi[0] < 0 || vi[0] >= a.V || vi[1] < 0 || vi[1] >= a.V || vi[2] < 0 || vi[2] >= a.V) {
        vi[0] = vi[1] = vi[2] = -1;
        return false;
    }
    n = find_mesh(a.first, a.nf, a.N, f);
    if (n < 0) return false;
    const float* P0 = a.verts + 3 * (int64_t)vi[0];
    const float* P1 = a.verts + 3 * (int64_t)vi[1];
    const float* P2 = a.verts + 3 * (int64_t)vi[2];
    R = make_rec(P0[0], P0[1], P0[2], P1[0], P1[1], P1[2], P2[0], P2[1], P2[2], a.rb, n, a.opts);
    vz[0] = P0[2];
    vz[1] = P1[2];
    vz[2] = P2[2];
    return R.ok();
}

__device__ __forceinline__ uint32_t vhash(int v) { return ((uint32_t)v * 2654435761u) >> (32 - 10); }

// Merges (vertex, grad3) into the workgroup's LDS table; falls back to a global
// atomic when the table is full.
__device__ __forceinline__ void lds_add(int* keys, float* vals, float* grad, int v, float x, float y, float z) {
    uint32_t h = vhash(v);
    for (int probe = 0; probe < kHash; ++probe) {
        int prev = atomicCAS(&keys[h], -1, v);
        if (prev == -1 || prev == v) {
            atomicAdd(&vals[3 * h + 0], x);
            atomicAdd(&vals[3 * h + 1], y);
            atomicAdd(&vals[3 * h + 2], z);
            return;
        }
        h = (h + 1) & (kHash - 1);
    }
    atomicAdd(grad + 3 * (int64_t)v + 0, x);
    atomicAdd(grad + 3 * (int64_t)v + 1, y);
    atomicAdd(grad + 3 * (int64_t)v + 2, z);
}

__global__ __launch_bounds__(kBwdBlock) void bwd_faces_kernel(BwdArgs a) {
    __shared__ int keys[kHash];
    __shared__ float vals[3 * kHash];
    for (int i = threadIdx.x; i < kHash; i += kBwdBlock) {
        keys[i] = -1;
        vals[3 * i] = vals[3 * i + 1] = vals[3 * i + 2] = 0.0f;
    }
    __syncthreads();
    const int64_t f = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x;
    FaceGrad g;
#pragma unroll
    for (int j = 0; j < 3; ++j) g.gx[j] = g.gy[j] = g.gzv[j] = 0.0f;
    int vi[3] = {-1, -1, -1};
    bool have = false;
    if (f < a.F) {
        FaceRec R;
        float vz[3];
        int n;
        if (load_face(a, f, R, vi, vz, n)) {
            int c0, c1, r0, r1;
            pix_range(R.bb.x, R.bb.y, a.W, c0, c1);
            pix_range(R.bb.z, R.bb.w, a.H, r0, r1);
            if (c1 >= c0 && r1 >= r0) {
                int area = (c1 - c0 + 1) * (r1 - r0 + 1);
                if (area > kBigArea) {
                    int pos = atomicAdd(&a.hdr[kHdrBigCount], 1);
                    a.big[pos] = (int)f;
                } else {
                    for (int r = r0; r <= r1; ++r)
                        for (int c = c0; c <= c1; ++c) scan_pixel(a, R, vz, (int)f, n, r, c, g);
                    have = true;
                }
            }
        }
    }
    if (have) {
#pragma unroll
        for (int j = 0; j < 3; ++j) lds_add(keys, vals, a.grad, vi[j], g.gx[j], g.gy[j], g.gzv[j]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHash; i += kBwdBlock) {
        int v = keys[i];
        if (v >= 0) {
            atomicAdd(a.grad + 3 * (int64_t)v + 0, vals[3 * i + 0]);
            atomicAdd(a.grad + 3 * (int64_t)v + 1, vals[3 * i + 1]);
            atomicAdd(a.grad + 3 * (int64_t)v + 2, vals[3 * i + 2]);
        }
    }
}

// Faces with large boxes: each workgroup takes the next listed face and its
// 256 threads share the pixel scan; the nine sums are reduced in LDS.  Every
// workgroup leaves once the list is exhausted.
__global__ __launch_bounds__(kBwdBlock) void bwd_big_faces_kernel(BwdArgs a) {
    __shared__ float red[9][kBwdBlock / 64];
    __shared__ int item_s;
    const int count = a.hdr[kHdrBigCount];
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&a.hdr[kHdrBigNext], 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= count) break;
        const int f = a.big[item];
        FaceRec R;
        int vi[3] = {-1, -1, -1};
        float vz[3];
        int n;
        FaceGrad g;
#pragma unroll
        for (int j = 0; j < 3; ++j) g.gx[j] = g.gy[j] = g.gzv[j] = 0.0f;
        bool ok = load_face(a, f, R, vi, vz, n);
        if (ok) {
            int c0, c1, r0, r1;
            pix_range(R.bb.x, R.bb.y, a.W, c0, c1);
            pix_range(R.bb.z, R.bb.w, a.H, r0, r1);
            const int w = c1 - c0 + 1;
            const int64_t area = (c1 >= c0 && r1 >= r0) ? (int64_t)w * (r1 - r0 + 1) : 0;
            for (int64_t q = threadIdx.x; q < area; q += kBwdBlock) {
                int r = r0 + (int)(q / w), c = c0 + (int)(q % w);
                scan_pixel(a, R, vz, f, n, r, c, g);
            }
        }
        float t[9] = {g.gx[0], g.gy[0], g.gzv[0], g.gx[1], g.gy[1], g.gzv[1], g.gx[2], g.gy[2], g.gzv[2]};
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            float v = t[j];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < 9 && ok) {
            float s = 0.0f;
            for (int w4 = 0; w4 < kBwdBlock / 64; ++w4) s += red[threadIdx.x][w4];
            int j = threadIdx.x / 3, x = threadIdx.x % 3;
            atomicAdd(a.grad + 3 * (int64_t)vi[j] + x, s);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Binned form.  Pass 1: one workgroup per bin reads the slots of the bin's
// pixels once (coalesced reads of pix_to_face and the gradients), maps each
// slot's face to a chunk index through an LDS hash table, and accumulates the
// nine coordinate sums per face in LDS as 64-bit fixed-point integers: integer
// LDS atomics cost next to nothing on this hardware and float LDS atomics a
// great deal (measured at config 4: 2.3 ms for the pass with float LDS
// atomics, 0.95 ms with integer ones), and the per-bin sums become exact and
// independent of the order of the additions.  The grid is 2^-S with
// S = 38 - 2 log2(bin size) (2^-32 at bin size 8); a term must lie below
// 2^min(51 - S, 62 - 2 log2(bin size) - S) (2^19 at bin size 8), where the
// conversion is exact and a face's at most bin_size^2 terms cannot overflow;
// a larger term (a sliver's geometric factor times a large gradient) goes to
// grad_verts directly with a float atomic.  Terms are rounded to the nearest
// grid point.  The pass records the largest face sum of the call (at the
// flush, off the hot loop); if it lies below 2^(18 - S) -- gradients so small
// that the grid holds them to fewer than 18 bits -- a second launch of the
// pass (the rescue) redoes the sums on a grid 2^30 times finer than that
// largest sum, after the vertex gradients are cleared again.  Normally the
// rescue launch only reads the recorded sum and exits.  A face's nine sums
// from a bin go to its own row partial[f][i] for the i-th bin of its range (no
// global atomic), and the row's byte in an (F, 4) mask is set.  Pass 2: one
// thread per face adds the rows the mask names and merges per vertex in LDS;
// one float atomic per (vertex, coordinate) per workgroup.  Faces spanning
// more than four bins take global atomics directly.
// ---------------------------------------------------------------------------
constexpr int kP1Threads = 256;
constexpr int kP1Chunk = 160;    // faces staged in LDS per pass over a bin's slots
static_assert(kP1Chunk <= kP1Threads, "a chunk's faces are gathered one per thread");
constexpr int kP1Table = 512;    // LDS hash entries (>= 2 * kP1Chunk)
constexpr int kP1Unroll = 4;     // slots per thread in one group of the bin's slots
constexpr int kP1Group = kP1Unroll * kP1Threads;  // slots the workgroup holds at once
constexpr int kMaxPartials = 4;  // (the row masks are read as one uchar4)

__device__ __forceinline__ uint32_t fhash(int f) { return ((uint32_t)f * 2654435761u) >> (32 - 9); }
static_assert(kP1Table == 512, "fhash yields 9 bits");

__device__ __forceinline__ void atomic_face(const BwdArgs& a, int f, const float* g9) {
    const int32_t* fv = a.faces + 3 * (int64_t)f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int v = fv[j];
        if (v < 0 || v >= a.V) continue;
#pragma unroll
        for (int x = 0; x < 3; ++x)
            if (g9[3 * j + x] != 0.0f) atomicAdd(a.grad + 3 * (int64_t)v + x, g9[3 * j + x]);
    }
}

// A face as the bin pass keeps it in LDS: the fields the slot recomputation
// reads (FaceRec without the mesh id and the box), 88 bytes.
struct Dbl2 {  // a pair of doubles at 8-byte alignment (double2 would pad the record to 96 bytes)
    double x, y;
};
struct BinRec {
    Dbl2 pa, ab, ac;
    double E;
    float az, dz1, dz2, invE, il0, il1, il2;
    int face;  // the face's id
};
static_assert(sizeof(BinRec) == 88, "bin record layout");

__device__ __forceinline__ void store_bin_rec(BinRec& d, const FaceRec& R, int f) {
    d.pa = {R.pa.x, R.pa.y};
    d.ab = {R.ab.x, R.ab.y};
    d.ac = {R.ac.x, R.ac.y};
    d.E = R.E;
    d.az = R.az;
    d.dz1 = R.dz1;
    d.dz2 = R.dz2;
    d.invE = R.invE;
    d.il0 = R.il0;
    d.il1 = R.il1;
    d.il2 = R.il2;
    d.face = f;
}

constexpr int kFixBits = 38;     // fixed-point grid 2^-(kFixBits - 2 log2(bin size))
constexpr int kRescueBits = 18;  // a largest face sum below 2^18 grid points triggers the rescue
constexpr int kRescueGrid = 2048;  // workgroups of the rescue launch

// v * 2^S rounded to the nearest integer (ties to even), as a two's-complement
// 64-bit integer, for abs(v) < 2^(51-S).  With M = 1.5 * 2^(52-S), the FP64
// sum v + M lies in M's binade, where one unit of the last place is 2^-S, so
// the addition itself rounds v to the grid and the difference of the two bit
// patterns is that rounded value: one conversion, one FP64 add and one 64-bit
// integer subtraction.  bits_m is the bit pattern of M.
__device__ __forceinline__ unsigned long long to_fix(float v, double m, unsigned long long bits_m) {
    return (unsigned long long)__double_as_longlong((double)v + m) - bits_m;
}

// Rescue condition from the recorded largest face sum (float bits, >= 0).
__device__ __forceinline__ bool needs_rescue(int tbits_max, int S) {
    return tbits_max > 0 && __int_as_float(tbits_max) < ldexpf(1.0f, kRescueBits - S);
}

// Pixel centre coordinate 1 - (2i+1)/n from the reciprocal rn = 1/n with one
// residual correction of the quotient: within one unit in the last place of
// the forward's correctly rounded division, at five FP64 operations instead
// of a division.  The backward only recomputes values of a face the forward
// already chose, so the last place of the pixel centre cannot change a
// decision that matters: it moves an edge function by about 1e-19.
__device__ __forceinline__ double pix_coord_rcp(int i, double n, double rn) {
    const double num = (double)(2 * i + 1);
    const double q0 = num * rn;
    const double r = fma(-q0, n, num);
    return 1.0 - fma(r, rn, q0);
}

// A thread's position in the bin's slot order (pixel-major, k fastest),
// advanced by kP1Threads slots at a time without divisions.
struct SlotWalk {
    int k, pr, pc;  // slot within the pixel, pixel row and column within the bin
    int dk, dpl;    // kP1Threads = dpl * K + dk
    int dr0, dc0;   // dpl pixels = dr0 rows + dc0 columns
    int dr1, dc1;   // dpl + 1 pixels
    __device__ __forceinline__ void init(int q, int K, int cols) {
        const int pl = q / K;
        k = q - pl * K;
        pr = pl / cols;
        pc = pl - pr * cols;
        dpl = kP1Threads / K;
        dk = kP1Threads - dpl * K;
        dr0 = dpl / cols;
        dc0 = dpl - dr0 * cols;
        dr1 = (dpl + 1) / cols;
        dc1 = (dpl + 1) - dr1 * cols;
    }
    __device__ __forceinline__ void next(int K, int cols) {
        k += dk;
        const bool carry = k >= K;
        k = carry ? k - K : k;
        pr += carry ? dr1 : dr0;
        pc += carry ? dc1 : dc0;
        const bool wrap = pc >= cols;
        pc = wrap ? pc - cols : pc;
        pr = wrap ? pr + 1 : pr;
    }
};

// The nine coordinate terms of one slot of face R (chunk index j) at pixel
// (row, col), added to the chunk's fixed-point sums.
struct FixGrid {
    float limit;              // terms at or above this go to grad_verts directly
    double m;                 // 1.5 * 2^(52 - S)
    unsigned long long bits;  // bit pattern of m
};
template <bool kOpts>
__device__ __forceinline__ void add_slot(const BwdArgs& a, const BinRec& R, int j, int row, int col, double dW,
                                         double rW, double dH, double rH, const SlotUp& up,
                                         unsigned long long* acci, const FixGrid& fx) {
    const float vz[3] = {R.az, R.az + R.dz1, R.az + R.dz2};
    FaceGrad g;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) g.gx[jj] = g.gy[jj] = g.gzv[jj] = 0.0f;
    Pix p;
    p.xf = p.yf = 0.0f;  // (the recomputation reads only the FP64 centre)
    p.x = pix_coord_rcp(col, dW, rW);
    p.y = pix_coord_rcp(row, dH, rH);
    slot_grad_up<BinRec, kOpts>(a, R, vz, p, up, g);
    const float g9[9] = {g.gx[0], g.gy[0], g.gzv[0], g.gx[1], g.gy[1], g.gzv[1], g.gx[2], g.gy[2], g.gzv[2]};
    float gmax = 0.0f;
#pragma unroll
    for (int x = 0; x < 9; ++x) gmax = fmaxf(gmax, fabsf(g9[x]));
    if (gmax < fx.limit) {
#pragma unroll
        for (int x = 0; x < 9; ++x) atomicAdd(&acci[9 * j + x], to_fix(g9[x], fx.m, fx.bits));
    } else {
        // a term too large for the fixed-point sums (never for sane inputs): straight to the vertex
#pragma unroll
        for (int x = 0; x < 9; ++x) {
            const float v = g9[x];
            if (fabsf(v) < fx.limit) {
                atomicAdd(&acci[9 * j + x], to_fix(v, fx.m, fx.bits));
            } else {
                const int vtx = a.faces[3 * (int64_t)R.face + x / 3];
                if (vtx >= 0 && vtx < a.V) atomicAdd(a.grad + 3 * (int64_t)vtx + x % 3, v);
            }
        }
    }
}

// Where face f's sums from bin (bx, by) go: its partial row f * 4 + i (i the
// bin's place in the face's range), -1 (vertex atomics: the range spans more
// than kMaxPartials bins) or -2 (nowhere: the face never counts, or the bin
// lies outside its range).
__device__ __forceinline__ int partial_row(const BwdArgs& a, const FaceRec& G, int f, int bx, int by) {
    int bx0, bx1, by0, by1;
    if (!face_bins(G, a.H, a.W, a.bs, bx0, bx1, by0, by1)) return -2;
    const int nb = (bx1 - bx0 + 1) * (by1 - by0 + 1);
    if (nb > kMaxPartials) return -1;
    if (bx < bx0 || bx > bx1 || by < by0 || by > by1) return -2;
    return f * kMaxPartials + (by - by0) * (bx1 - bx0 + 1) + (bx - bx0);
}

// Writes a chunk face's sums (or sends them to the vertices) and marks the
// partial row as written; tracks the workgroup's largest sum.
__device__ __forceinline__ void flush_face(const BwdArgs& a, const unsigned long long* acc9, int dst, int face, int S,
                                           bool track, int* smax) {
    if (dst == -2) return;
    float g9[9];
    float fmx = 0.0f;
#pragma unroll
    for (int x = 0; x < 9; ++x) {
        g9[x] = (float)ldexp((double)(long long)acc9[x], -S);
        fmx = fmaxf(fmx, fabsf(g9[x]));
    }
    // non-negative floats order as their bit patterns
    if (track && fmx > 0.0f) atomicMax(smax, __float_as_int(fmx));
    if (dst >= 0) {
        float* out = a.partial + (int64_t)dst * 9;
#pragma unroll
        for (int x = 0; x < 9; ++x) out[x] = g9[x];
        a.pmask[dst] = 1;
    } else {
        atomic_face(a, face, g9);
    }
}

// rescue = 0: the pass, recording its largest face sum; rescue = 1: the
// rescue pass, which exits unless that sum calls for it.  kOpts: the call
// has perspective-correct or clipped barycentrics (an instance of its own, so
// that their register needs do not lower the occupancy of the plain one).
//
// Two ways through a bin.  The direct way (a bin of at most kP1Group slots
// whose slots name at most kP1Chunk distinct faces, nearly every bin): the
// slots' face ids and upstream gradients are requested at once, the distinct
// ids go into the LDS hash table as they arrive (the inserting lane numbers
// the face), their records are gathered -- while the gradients are still in
// flight -- and every slot is recomputed once.  Only the faces the slots name
// are gathered, so a crowded bin (silhouettes) costs no more than a quiet one,
// and the bin's list is not read.  Slot ids outside [0, F), of a face that
// never counts or of another image are ignored.  The listed way (any other
// bin): the bin's list is taken in chunks of kP1Chunk faces, each chunk's
// records and hash table built, and every slot of the bin looked up in it.
template <bool kOpts, bool kLoop>
__global__ __launch_bounds__(kP1Threads) __attribute__((amdgpu_waves_per_eu(5, 8)))
void bwd_bins_kernel(BwdArgs a, int rescue) {
    __shared__ BinRec srec[kP1Chunk];
    __shared__ unsigned long long acci[kP1Chunk * 9];
    __shared__ int tkey[kP1Table];
    __shared__ short tval[kP1Table];  // the key's face: its chunk index (-1: held over to the listed way)
    __shared__ int sdst[kP1Chunk];    // partial_row of each chunk face
    __shared__ int ucount, ufail;
    int lgbs = 0;
    while ((1 << lgbs) < a.bs) ++lgbs;
    int S = kFixBits - 2 * lgbs;  // grid exponent of the sums
    if (rescue) {
        const int tb = a.hdr[kHdrTermMax];
        if (!needs_rescue(tb, S)) return;
        // the largest sum (< 2^eb) on 2^30 grid points
        S = 30 - (((tb >> 23) & 0xff) - 126);
    }
    // terms below the limit: the conversion is exact, and a face's at most
    // bs^2 of them stay below 2^62 on the grid
    FixGrid fx;
    fx.limit = ldexpf(1.0f, min(51, 62 - 2 * lgbs) - S);
    fx.m = ldexp(1.5, 52 - S);
    fx.bits = (unsigned long long)__double_as_longlong(fx.m);
    __shared__ int smax;  // largest abs face sum of the workgroup (float bits)
    if (!bins_usable(a)) return;
    if (threadIdx.x == 0) smax = 0;  // (ordered before every update by the first bin's barriers)
    const bool track = !rescue;
    const int per_img = a.nby * a.nbx;
    const int64_t nbins = (int64_t)a.N * per_img;
    // kLoop: a grid smaller than the bin count (the rescue launch) walks the
    // bins; otherwise the grid is one workgroup per bin, each XCD taking a
    // contiguous range of bins (neighbouring bins gather mostly the same
    // face records; xcd_item).  Either way the first bin is < nbins.
    int64_t bin = kLoop ? (int64_t)blockIdx.x : xcd_item(blockIdx.x, nbins);
    do {
        const int n = (int)(bin / per_img);
        const int rem = (int)(bin - (int64_t)n * per_img);
        const int by = rem / a.nbx, bx = rem - (rem / a.nbx) * a.nbx;
        const int r0 = by * a.bs, c0 = bx * a.bs;
        const int rows = min(a.bs, a.H - r0), cols = min(a.bs, a.W - c0);
        const int nslots = rows * cols * a.K;
        // slot (pr, pc, k) of the bin is pix_to_face[sbase + (pr * W + pc) * K + k]
        const int64_t sbase = (((int64_t)n * a.H + r0) * a.W + c0) * a.K;
        const double dW = (double)a.W, dH = (double)a.H, rW = 1.0 / dW, rH = 1.0 / dH;

        if (nslots <= kP1Group) {
            // ---- the direct way
            SlotWalk w;
            w.init(threadIdx.x, a.K, cols);
            int fq[kP1Unroll], rq[kP1Unroll], cq[kP1Unroll];
#pragma unroll
            for (int u = 0; u < kP1Unroll; ++u) {
                const int q = u * kP1Threads + threadIdx.x;
                rq[u] = r0 + w.pr;
                cq[u] = c0 + w.pc;
                int f = -1;
                if (q < nslots)
                    f = __builtin_nontemporal_load(a.p2f + sbase + (int64_t)(w.pr * a.W + w.pc) * a.K + w.k);
                fq[u] = (f >= 0 && f < a.F) ? f : -1;
                w.next(a.K, cols);
            }
            for (int i = threadIdx.x; i < kP1Table; i += kP1Threads) tkey[i] = -1;
            if (threadIdx.x == 0) {
                ucount = 0;
                ufail = 0;
            }
            SlotUp up[kP1Unroll];
            {
                SlotWalk w2;
                w2.init(threadIdx.x, a.K, cols);
#pragma unroll
                for (int u = 0; u < kP1Unroll; ++u) {
                    up[u] = SlotUp{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                    if (fq[u] >= 0) up[u] = load_up(a, sbase + (int64_t)(w2.pr * a.W + w2.pc) * a.K + w2.k);
                    w2.next(a.K, cols);
                }
            }
            __syncthreads();
            // distinct faces into the table; the lane that inserts a face numbers it
#pragma unroll
            for (int u = 0; u < kP1Unroll; ++u) {
                const int f = fq[u];
                if (f < 0) continue;
                uint32_t h = fhash(f);
                bool placed = false;
                for (int probe = 0; probe < kP1Table; ++probe) {
                    const int prev = atomicCAS(&tkey[h], -1, f);
                    if (prev == -1) {
                        const int j = atomicAdd(&ucount, 1);
                        tval[h] = (short)(j < kP1Chunk ? j : -1);
                        placed = true;
                        break;
                    }
                    if (prev == f) {
                        placed = true;
                        break;
                    }
                    h = (h + 1) & (kP1Table - 1);
                }
                if (!placed) ufail = 1;  // (a full table: the listed way takes the bin)
            }
            __syncthreads();
            const int U = ucount;
            if (U <= kP1Chunk && !ufail) {
                // records of the named faces, one thread per table entry
                for (int i = threadIdx.x; i < kP1Table; i += kP1Threads) {
                    const int f = tkey[i];
                    if (f < 0) continue;
                    const int j = tval[i];
                    const FaceRec& G = a.recs[f];
                    store_bin_rec(srec[j], G, f);
                    const bool ok = G.ok() && G.mesh() == n;
                    if (!ok) srec[j].face = -1;
                    sdst[j] = ok ? partial_row(a, G, f, bx, by) : -2;
#pragma unroll
                    for (int x = 0; x < 9; ++x) acci[9 * j + x] = 0ull;
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < kP1Unroll; ++u) {
                    const int f = fq[u];
                    if (f < 0) continue;
                    uint32_t h = fhash(f);
                    for (int probe = 0; probe < kP1Table && tkey[h] != f; ++probe) h = (h + 1) & (kP1Table - 1);
                    const int j = tval[h];  // (every named face was placed)
                    const BinRec R = srec[j];
                    if (R.face < 0) continue;
                    add_slot<kOpts>(a, R, j, rq[u], cq[u], dW, rW, dH, rH, up[u], acci, fx);
                }
                __syncthreads();
                for (int j = threadIdx.x; j < U; j += kP1Threads)
                    flush_face(a, &acci[9 * j], sdst[j], srec[j].face, S, track, &smax);
                __syncthreads();
                continue;
            }
            // (every thread has read ucount and ufail: the listed way may now reuse the table)
        }

        // ---- the listed way
        const int cnt = min(a.counts[bin], a.M);
        const int* list = a.lists + bin * a.M;
        for (int base = 0; base < cnt; base += kP1Chunk) {
            const int m = min(kP1Chunk, cnt - base);
            for (int i = threadIdx.x; i < kP1Table; i += kP1Threads) tkey[i] = -1;
            for (int i = threadIdx.x; i < m * 9; i += kP1Threads) acci[i] = 0ull;
            __syncthreads();
            const int t = threadIdx.x;
            if (t < m) {
                const int j = t;
                const int f = list[base + j];
                const FaceRec& G = a.recs[f];
                store_bin_rec(srec[j], G, f);
                sdst[j] = partial_row(a, G, f, bx, by);
                uint32_t h = fhash(f);
                for (int probe = 0; probe < kP1Table; ++probe) {
                    if (atomicCAS(&tkey[h], -1, f) == -1) {
                        tval[h] = (short)j;
                        break;
                    }
                    h = (h + 1) & (kP1Table - 1);
                }
            }
            __syncthreads();
            SlotWalk w;
            w.init(threadIdx.x, a.K, cols);
            for (int q0 = 0; q0 < nslots; q0 += kP1Group) {
                int fq[kP1Unroll], rq[kP1Unroll], cq[kP1Unroll];
                int64_t sq[kP1Unroll];
#pragma unroll
                for (int u = 0; u < kP1Unroll; ++u) {
                    const int q = q0 + u * kP1Threads + threadIdx.x;
                    fq[u] = -1;
                    rq[u] = r0 + w.pr;
                    cq[u] = c0 + w.pc;
                    sq[u] = 0;
                    if (q < nslots) {
                        sq[u] = sbase + ((int64_t)(w.pr * a.W + w.pc) * a.K + w.k);
                        fq[u] = __builtin_nontemporal_load(a.p2f + sq[u]);
                    }
                    w.next(a.K, cols);
                }
#pragma unroll
                for (int u = 0; u < kP1Unroll; ++u) {
                    const int f = fq[u];
                    if (f < 0) continue;
                    int j = -1;
                    uint32_t h = fhash(f);
                    for (int probe = 0; probe < kP1Table; ++probe) {
                        const int key = tkey[h];
                        if (key == f) {
                            j = tval[h];
                            break;
                        }
                        if (key == -1) break;
                        h = (h + 1) & (kP1Table - 1);
                    }
                    if (j < 0) continue;
                    add_slot<kOpts>(a, srec[j], j, rq[u], cq[u], dW, rW, dH, rH, load_up(a, sq[u]), acci, fx);
                }
            }
            __syncthreads();
            // flush: one partial per listed face (written and marked, zero or not)
            if (t < m) flush_face(a, &acci[9 * t], sdst[t], srec[t].face, S, track, &smax);
            __syncthreads();
        }
        __syncthreads();  // (a bin without chunks has no barrier of its own)
    } while (kLoop && (bin += gridDim.x) < nbins);
    if (track && threadIdx.x == 0) {
        // the call's largest face sum: one global word, so a workgroup only
        // updates it when its own maximum is larger than what it reads there
        // (same-address atomics from every wave would serialise)
        const int mine = smax;
        if (mine > 0 && mine > __hip_atomic_load(&a.hdr[kHdrTermMax], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&a.hdr[kHdrTermMax], mine);
    }
}

// Clears grad_verts before the rescue pass, when the recorded largest sum calls for it.
__global__ void bwd_rescue_clear_kernel(BwdArgs a) {
    int lgbs = 0;
    while ((1 << lgbs) < a.bs) ++lgbs;
    if (!needs_rescue(a.hdr[kHdrTermMax], kFixBits - 2 * lgbs)) return;
    const int64_t n = a.V * 3;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a.grad[i] = 0.0f;
}


// Pass 2: one thread per face adds the partial rows this call wrote for it
// and merges the result per vertex in an LDS hash table, as 64-bit fixed point
// (integer LDS atomics; float ones are slow on this hardware); each table
// entry then issues one float atomic per coordinate.  The grid follows the
// largest row the pass recorded (below 2^e): a face's sum of at most four rows
// stays below 2^(e+2) and a vertex takes at most kBwdBlock faces of the
// workgroup, below 2^(e+10), so the grid 2^(e-48) keeps every sum below 2^58
// and every term inside to_fix's exact range.
__global__ __launch_bounds__(kBwdBlock) void bwd_face_sum_kernel(BwdArgs a) {
    __shared__ int keys[kHash];
    __shared__ unsigned long long vals[3 * kHash];
    if (!bins_usable(a)) return;
    const int tb = a.hdr[kHdrTermMax];
    if (tb <= 0) return;  // every row is zero
    const int e = ((tb >> 23) & 0xff) - 126;
    const int S = 48 - e;
    const double fm = ldexp(1.5, 52 - S);
    const unsigned long long fbits = (unsigned long long)__double_as_longlong(fm);
    for (int i = threadIdx.x; i < kHash; i += kBwdBlock) {
        keys[i] = -1;
        vals[3 * i] = vals[3 * i + 1] = vals[3 * i + 2] = 0ull;
    }
    __syncthreads();
    const int64_t f = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x;
    const bool overflowed = (a.hdr[kHdrStatus] & kStatOverflow) != 0;
    if (f < a.F && !overflowed) {
        // the rows this call wrote (none for a face whose sums went to the
        // vertices directly, or that no slot names)
        const uchar4 mk = *reinterpret_cast<const uchar4*>(a.pmask + f * kMaxPartials);
        if (mk.x | mk.y | mk.z | mk.w) {
            const bool wr[kMaxPartials] = {mk.x != 0, mk.y != 0, mk.z != 0, mk.w != 0};
            float g9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            const float* src = a.partial + f * kMaxPartials * 9;
#pragma unroll
            for (int i = 0; i < kMaxPartials; ++i) {
                if (!wr[i]) continue;
#pragma unroll
                for (int x = 0; x < 9; ++x) g9[x] += src[9 * i + x];
            }
            const int32_t* fv = a.faces + 3 * f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int v = fv[j];
                if (v < 0 || v >= a.V) continue;
                uint32_t h = vhash(v);
                bool placed = false;
                for (int probe = 0; probe < kHash; ++probe) {
                    const int prev = atomicCAS(&keys[h], -1, v);
                    if (prev == -1 || prev == v) {
#pragma unroll
                        for (int x = 0; x < 3; ++x) atomicAdd(&vals[3 * h + x], to_fix(g9[3 * j + x], fm, fbits));
                        placed = true;
                        break;
                    }
                    h = (h + 1) & (kHash - 1);
                }
                if (!placed) {
#pragma unroll
                    for (int x = 0; x < 3; ++x) atomicAdd(a.grad + 3 * (int64_t)v + x, g9[3 * j + x]);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHash; i += kBwdBlock) {
        const int v = keys[i];
        if (v >= 0) {
#pragma unroll
            for (int x = 0; x < 3; ++x)
                atomicAdd(a.grad + 3 * (int64_t)v + x, (float)ldexp((double)(long long)vals[3 * i + x], -S));
        }
    }
}

// Zeroes grad_verts (n3v floats) and the row masks (nmask words), and the
// recorded largest face sum.
__global__ void bwd_prep_kernel(float* __restrict__ grad, int64_t n3v, int* __restrict__ mask, int64_t nmask,
                                int* __restrict__ term) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < n3v; i += stride) grad[i] = 0.0f;
    for (int64_t i = i0; i < nmask; i += stride) mask[i] = 0;
    if (i0 == 0) *term = 0;
}

hipError_t launch_backward(const float* verts, int64_t V, const int32_t* faces, int64_t F, const int64_t* first,
                           const int64_t* nf, int N, int H, int W, int K, float blur, int opts, int bs, int M,
                           const int32_t* p2f, const float* gz, const float* gb, const float* gd, float* grad,
                           int* hdr, FaceRec* recs, int* counts, int* lists, float* partial, int* big,
                           bool reuse, const BinSig& sig, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    reuse = reuse && bs > 0;
    hipError_t e = hipSuccess;
    // the binned form clears grad_verts together with its row masks (below)
    if (bs == 0 || F == 0) {
        e = launch_fill_f32(grad, V * 3, 0.0f, s);
        if (e != hipSuccess) return e;
    }
    if (!reuse) {
        e = launch_fill_i32(hdr, kHdrWords, 0, s);
        if (e != hipSuccess) return e;
    }
    if (F == 0) return hipSuccess;
    BwdArgs a;
    a.verts = verts;
    a.faces = faces;
    a.first = first;
    a.nf = nf;
    a.p2f = p2f;
    a.gz = gz;
    a.gb = gb;
    a.gd = gd;
    a.grad = grad;
    a.hdr = hdr;
    a.big = big;
    a.V = V;
    a.F = F;
    a.N = N;
    a.H = H;
    a.W = W;
    a.K = K;
    a.rb = sqrtf(blur);
    a.opts = opts;
    a.recs = recs;
    a.counts = counts;
    a.lists = lists;
    a.partial = partial;
    a.pmask = reinterpret_cast<unsigned char*>(big);
    a.bs = bs;
    a.nby = bs > 0 ? (H + bs - 1) / bs : 0;
    a.nbx = bs > 0 ? (W + bs - 1) / bs : 0;
    a.M = M;
    a.reuse = reuse ? 1 : 0;
    a.sig = sig;
    if (bs > 0) {
        // the same face setup and binning as the forward (unless the forward's
        // are reused), then the two passes
        if (!reuse) {
            e = launch_face_setup(verts, V, faces, F, first, nf, N, a.rb, opts, recs, hdr, s);
            if (e != hipSuccess) return e;
            e = launch_binning(recs, F, N, H, W, bs, M, counts, lists, hdr, s);
            if (e != hipSuccess) return e;
        }
        const int64_t nbins = (int64_t)N * a.nby * a.nbx;
        // grad_verts, the row masks (no partial row is written yet: F x 4 mask
        // bytes = F words) and the recorded largest sum, in one launch
        hipLaunchKernelGGL(bwd_prep_kernel, dim3(1024), dim3(256), 0, s, grad, V * 3, big, F, hdr + kHdrTermMax);
        if (eb) (void)hipEventRecord(eb, s);
        const bool o = (opts & (kOptPersp | kOptClip)) != 0;
        auto bins = o ? bwd_bins_kernel<true, false> : bwd_bins_kernel<false, false>;
        auto rescue = o ? bwd_bins_kernel<true, true> : bwd_bins_kernel<false, true>;
        hipLaunchKernelGGL(bins, dim3((unsigned)nbins), dim3(kP1Threads), 0, s, a, 0);
        hipLaunchKernelGGL(bwd_rescue_clear_kernel, dim3(256), dim3(256), 0, s, a);
        // the rescue launch normally exits at once: a small grid that walks the bins when it does not
        hipLaunchKernelGGL(rescue, dim3((unsigned)(nbins < kRescueGrid ? nbins : kRescueGrid)), dim3(kP1Threads), 0,
                           s, a, 1);
        hipLaunchKernelGGL(bwd_face_sum_kernel, dim3((unsigned)((F + kBwdBlock - 1) / kBwdBlock)), dim3(kBwdBlock), 0,
                           s, a);
        if (ee) (void)hipEventRecord(ee, s);
        return hipGetLastError();
    }
    if (eb) (void)hipEventRecord(eb, s);
    hipLaunchKernelGGL(bwd_faces_kernel, dim3((unsigned)((F + kBwdBlock - 1) / kBwdBlock)), dim3(kBwdBlock), 0, s, a);
    hipLaunchKernelGGL(bwd_big_faces_kernel, dim3(512), dim3(kBwdBlock), 0, s, a);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

}  // namespace rast
