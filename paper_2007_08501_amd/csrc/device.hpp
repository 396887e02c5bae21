// device.hpp -- per-face and per-pixel arithmetic of the rasterizer for gfx950.
//
// Everything that decides whether a face counts for a pixel, and the values
// written for it, lives here so that the single-pass and the binned forward
// and the backward evaluate every (pixel, face) pair with the same
// instructions (the library is built with -ffp-contract=off, so the compiler
// cannot fuse differently in different kernels).
//
// Accuracy.  Faces seen edge-on (near a silhouette) project to slivers whose
// doubled area E is tiny, and a barycentric w_i = e_i / E amplifies any error
// of the edge function e_i by 1/E.  The edge functions are therefore formed
// in FP64 from exact operands: the vertex offsets b - a, c - a of FP32
// vertices and the pixel offset p - a are exact in FP64, leaving one rounding
// of 2^-53 per product, far below what an FP32 barycentric can show.  On
// CDNA vector FP64 issues at the same rate as non-packed FP32, so this costs
// fewer instructions than compensated FP32 arithmetic.  Everything else
// (depth, distances, the backward's chain rule) is FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rast {

constexpr double kEpsArea = 1e-8;  // faces with abs(2 * signed area) below this never count
constexpr int kTile = 8;           // forward work unit: 8x8 pixels = one wave64

// Rasterizer options (the bits of the ABI's options / flags words).
constexpr int kOptPersp = 0x100;  // perspective-correct barycentrics
constexpr int kOptClip = 0x200;   // barycentrics clipped to [0, 1] and renormalised
constexpr int kOptCull = 0x400;   // back faces (E > 0) never count
constexpr int kOptMask = kOptPersp | kOptClip | kOptCull;

// Workspace header (int32 words); the header occupies the first 256 bytes.
enum : int {
    kHdrStatus = 0,     // sticky status bits (kStatOverflow | kStatMesh)
    kHdrMaxCount = 1,   // largest bin count seen
    kHdrWorkNext = 2,   // persistent scheduler: next work item
    kHdrWorkTotal = 3,  // persistent scheduler: number of work items
    kHdrBigCount = 8,   // backward: number of faces with large pixel boxes
    kHdrBigNext = 9,    // backward: next large face to scan
    kHdrTermMax = 10,   // backward: largest abs face sum of the binned pass (float bits)
    kHdrSig = 16,       // kSigWords words: what the last forward binned (see BinSig)
    kHdrWords = 64,
};
enum : int { kStatOverflow = 1, kStatMesh = 2, kStatReuse = 4 };

// What a binned forward leaves in its workspace for a backward that reuses
// its face records and bins: a marker, F, N, H, W, bin size, capacity and
// the bit pattern of the blur radius.
constexpr int kSigWords = 8;
constexpr int kSigMarker = 0x52535447;
constexpr int kPtSigMarker = 0x50545347;  // point-cloud workspaces
struct BinSig {
    int w[kSigWords];
};

// Pixel centre in NDC: x = 1 - (2c+1)/W, y = 1 - (2r+1)/H.  The FP32 value
// (exact for power-of-two sizes) is used for box tests and tile extents, the
// FP64 value for edge functions.
__device__ __forceinline__ float pix_x(int c, int W) { return 1.0f - (float)(2 * c + 1) / (float)W; }
__device__ __forceinline__ float pix_y(int r, int H) { return 1.0f - (float)(2 * r + 1) / (float)H; }

struct Pix {
    float xf, yf;  // FP32 centre
    double x, y;   // FP64 centre
};
__device__ __forceinline__ Pix make_pix(int r, int c, int H, int W) {
    Pix p;
    p.xf = pix_x(c, W);
    p.yf = pix_y(r, H);
    p.x = 1.0 - (double)(2 * c + 1) / (double)W;
    p.y = 1.0 - (double)(2 * r + 1) / (double)H;
    return p;
}

// Per-face record, 112 bytes, built once per call by the setup kernel.
struct FaceRec {
    double2 pa;  // vertex a (x, y)
    double2 ab;  // b - a (exact)
    double2 ac;  // c - a (exact)
    double E;    // doubled signed area cross(b - a, c - a)
    float az;    // depth of a
    int mesh_;   // mesh (image) id; -1 = the face never counts
    float dz1, dz2;  // bz - az, cz - az
    float invE;      // 1 / E rounded to FP32
    float il0;       // 1 / |b - a|^2
    float il1, il2;  // 1 / |c - b|^2, 1 / |a - c|^2
    float pad_[2];
    float4 bb;   // xmin, xmax, ymin, ymax: xy box grown by sqrt(blur) plus a pad;
                 // empty (+inf, -inf) for faces that never count
    __device__ __forceinline__ int mesh() const { return mesh_; }
    __device__ __forceinline__ bool ok() const { return mesh_ >= 0; }
};

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// Builds the record of face (a, b, c).  rb = sqrt(blur_radius) in NDC units.
// Under the options a back face (E > 0: clockwise as the image is displayed,
// +x being to the left) or, with the perspective correction, a face with a
// vertex at z <= 0 never counts.
__device__ __forceinline__ FaceRec make_rec(float ax, float ay, float az, float bx, float by, float bz, float cx,
                                            float cy, float cz, float rb, int mesh, int opts = 0) {
    FaceRec R;
    R.pa = make_double2(ax, ay);
    R.ab = make_double2((double)bx - (double)ax, (double)by - (double)ay);
    R.ac = make_double2((double)cx - (double)ax, (double)cy - (double)ay);
    R.E = R.ab.x * R.ac.y - R.ab.y * R.ac.x;
    bool ok = mesh >= 0 && fabs(R.E) >= kEpsArea && finite3(ax, ay, az) && finite3(bx, by, bz) &&
              finite3(cx, cy, cz);
    if ((opts & kOptCull) && R.E > 0.0) ok = false;
    if ((opts & kOptPersp) && !(az > 0.0f && bz > 0.0f && cz > 0.0f)) ok = false;
    R.az = az;
    R.mesh_ = ok ? mesh : -1;
    R.dz1 = bz - az;
    R.dz2 = cz - az;
    R.invE = ok ? (float)(1.0 / R.E) : 0.0f;
    // edge lengths from the exact FP64 edge vectors (c - b = (c - a) - (b - a) is exact too)
    const double bcx = R.ac.x - R.ab.x, bcy = R.ac.y - R.ab.y;
    R.il0 = ok ? (float)(1.0 / (R.ab.x * R.ab.x + R.ab.y * R.ab.y)) : 0.0f;
    R.il1 = ok ? (float)(1.0 / (bcx * bcx + bcy * bcy)) : 0.0f;
    R.il2 = ok ? (float)(1.0 / (R.ac.x * R.ac.x + R.ac.y * R.ac.y)) : 0.0f;
    R.pad_[0] = R.pad_[1] = 0.0f;
    if (ok) {
        // The pad covers the FP32 error of the distance test: a pixel whose
        // FP32 squared distance is < blur is never farther than rb*(1+1e-6)+1e-7.
        float pad = rb * 1e-4f + 1e-6f;
        float g = rb + pad;
        R.bb = make_float4(fminf(ax, fminf(bx, cx)) - g, fmaxf(ax, fmaxf(bx, cx)) + g,
                           fminf(ay, fminf(by, cy)) - g, fmaxf(ay, fmaxf(by, cy)) + g);
    } else {
        R.bb = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    }
    return R;
}

// The evaluation below takes any record with FaceRec's geometry fields (pa,
// ab, ac, E, az, dz1, dz2, invE, il0, il1, il2): the same source expressions,
// built without contraction, give bit-identical results for every record
// type.
//
// Everything the forward writes for one (pixel, face) pair, and what the
// backward needs besides.
struct Eval {
    float w0, w1, w2;  // barycentrics
    float z;
    float d2;      // squared distance to the nearest boundary point
    float u;       // parameter of the nearest point on the nearest edge
    int edge;      // nearest edge: 0 = (a,b), 1 = (b,c), 2 = (c,a); lowest index on ties
    bool inside;   // all three barycentrics > 0
    float sx, sy;  // p - a (rounded): the pixel relative to vertex a
    double dx, dy; // p - a, exact
    float f0, f1, f2;  // the edge functions e0, e1, e2 rounded to FP32
};

// Barycentrics, z and inside-ness of pixel p in face R.
//   e1 = cross(p - a, c - a), e2 = cross(b - a, p - a), e0 = E - e1 - e2
// (the same three sub-triangle areas as cross(b-p, c-p), cross(c-p, a-p) and
// cross(a-p, b-p)), each FP64; w_i = e_i / E.  The pixel is inside when all
// three w_i are positive (each w_i has the sign of e_i / E).
template <class Rec>
__device__ __forceinline__ void eval_bary(const Rec& R, const Pix& p, Eval& o) {
    const double dx = p.x - R.pa.x, dy = p.y - R.pa.y;
    const double e1 = fma(dx, R.ac.y, -(dy * R.ac.x));
    const double e2 = fma(R.ab.x, dy, -(R.ab.y * dx));
    const double e0 = (R.E - e1) - e2;
    o.f0 = (float)e0;
    o.f1 = (float)e1;
    o.f2 = (float)e2;
    o.w0 = o.f0 * R.invE;
    o.w1 = o.f1 * R.invE;
    o.w2 = o.f2 * R.invE;
    // z = w0 az + w1 bz + w2 cz, rearranged with w0 = 1 - w1 - w2 so that the
    // large common depth az is added last
    o.z = fmaf(o.w2, R.dz2, o.w1 * R.dz1) + R.az;
    o.inside = fminf(o.w0, fminf(o.w1, o.w2)) > 0.0f;
    o.sx = (float)dx;
    o.sy = (float)dy;
    o.dx = dx;
    o.dy = dy;
}

// Squared distances from the pixel to the three boundary segments.  For
// segment P->Q with t = (p - P).(Q - P) / |Q - P|^2 the nearest point is P
// (t <= 0), Q (t >= 1) or the foot of the perpendicular, at squared distance
// e^2 / |Q - P|^2 from the edge function e of that edge (2 * the area of
// (P, Q, p)), which is formed in FP64 and so keeps its accuracy however
// close the pixel is to the line.
struct EdgeD {
    float d[3];  // squared distance per edge
    float t[3];  // unclamped parameter per edge
};
template <class Rec>
__device__ __forceinline__ void eval_edges(const Rec& R, const Eval& b, EdgeD& o) {
    const float abx = (float)R.ab.x, aby = (float)R.ab.y, acx = (float)R.ac.x, acy = (float)R.ac.y;
    // the pixel's offsets from the three vertices, each formed exactly in
    // FP64 and rounded once: a difference of rounded offsets would lose the
    // relative accuracy of the distance to b or c close to that vertex
    const float pax = b.sx, pay = b.sy;                                   // p - a
    const float pbx = (float)(b.dx - R.ab.x), pby = (float)(b.dy - R.ab.y);  // p - b
    const float pcx = (float)(b.dx - R.ac.x), pcy = (float)(b.dy - R.ac.y);  // p - c
    const float bcx = acx - abx, bcy = acy - aby;    // c - b
    const float da = fmaf(pax, pax, pay * pay), db = fmaf(pbx, pbx, pby * pby), dc = fmaf(pcx, pcx, pcy * pcy);
    o.t[0] = fmaf(pax, abx, pay * aby) * R.il0;
    o.t[1] = fmaf(pbx, bcx, pby * bcy) * R.il1;
    o.t[2] = -fmaf(pcx, acx, pcy * acy) * R.il2;
    const float q0 = b.f2 * b.f2 * R.il0, q1 = b.f0 * b.f0 * R.il1, q2 = b.f1 * b.f1 * R.il2;
    o.d[0] = o.t[0] <= 0.0f ? da : (o.t[0] >= 1.0f ? db : q0);
    o.d[1] = o.t[1] <= 0.0f ? db : (o.t[1] >= 1.0f ? dc : q1);
    o.d[2] = o.t[2] <= 0.0f ? dc : (o.t[2] >= 1.0f ? da : q2);
}

// Nearest edge (lowest index on ties), its squared distance and clamped parameter.
template <class Rec>
__device__ __forceinline__ void eval_dist(const Rec& R, Eval& o) {
    EdgeD ed;
    eval_edges(R, o, ed);
    float d = ed.d[0], t = ed.t[0];
    int e = 0;
    if (ed.d[1] < d) { d = ed.d[1]; e = 1; t = ed.t[1]; }
    if (ed.d[2] < d) { d = ed.d[2]; e = 2; t = ed.t[2]; }
    o.d2 = d;
    o.edge = e;
    o.u = fminf(fmaxf(t, 0.0f), 1.0f);
}

template <class Rec>
__device__ __forceinline__ void eval_full(const Rec& R, const Pix& p, Eval& o) {
    eval_bary(R, p, o);
    eval_dist(R, o);
}

__device__ __forceinline__ bool in_bbox(const FaceRec& R, const Pix& p) {
    return p.xf >= R.bb.x && p.xf <= R.bb.y && p.yf >= R.bb.z && p.yf <= R.bb.w;
}

// The options' barycentrics and depth from the raw ones (az the depth of
// vertex a, dz1 / dz2 those of b and c relative to it): with the
// perspective correction w_i <- (w_i / z_i) / sum_j (w_j / z_j), then with
// clipping w_i <- max(w_i, 0) / sum_j max(w_j, 0); z is interpolated with the
// result.  False when the options exclude the pair (a correction whose
// denominator is not positive).
__device__ __forceinline__ bool apply_opts(int opts, float az, float dz1, float dz2, float& w0, float& w1, float& w2,
                                           float& z) {
    if (opts & kOptPersp) {
        const float u0 = w0 / az, u1 = w1 / (az + dz1), u2 = w2 / (az + dz2);
        const float D = u0 + u1 + u2;
        if (!(D > 0.0f)) return false;
        w0 = u0 / D;
        w1 = u1 / D;
        w2 = u2 / D;
    }
    if (opts & kOptClip) {
        const float m0 = fmaxf(w0, 0.0f), m1 = fmaxf(w1, 0.0f), m2 = fmaxf(w2, 0.0f);
        const float M = m0 + m1 + m2;
        if (!(M > 0.0f)) return false;
        w0 = m0 / M;
        w1 = m1 / M;
        w2 = m2 / M;
    }
    z = fmaf(w2, dz2, w1 * dz1) + az;
    return true;
}

// Does face R count for pixel p, given that p lies in R's grown box?  On
// success z is its depth (under the options, if any).
template <class Rec>
__device__ __forceinline__ bool face_counts_in_box(const Rec& R, const Pix& p, float blur, float& z, int opts = 0) {
    Eval b;
    eval_bary(R, p, b);
    z = b.z;
    if (opts & (kOptPersp | kOptClip)) {
        float w0 = b.w0, w1 = b.w1, w2 = b.w2;
        if (!apply_opts(opts, R.az, R.dz1, R.dz2, w0, w1, w2, z)) return false;
    }
    if (!(z >= 0.0f)) return false;
    if (b.inside) return true;
    EdgeD ed;
    eval_edges(R, b, ed);
    return fminf(ed.d[0], fminf(ed.d[1], ed.d[2])) < blur;
}

// Mesh of face f: the last n with first[n] <= f, if f lies in its range.
__device__ __forceinline__ int find_mesh(const int64_t* __restrict__ first, const int64_t* __restrict__ nf, int N,
                                         int64_t f) {
    int lo = 0, hi = N - 1, ans = -1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        if (first[mid] <= f) {
            ans = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    if (ans >= 0 && f < first[ans] + nf[ans]) return ans;
    return -1;
}

// Inclusive pixel range [lo, hi] whose centres may fall in [vmin, vmax] along
// one axis of `size` pixels (centre of pixel i at 1 - (2i+1)/size); empty when
// hi < lo.  The FP32 evaluation of the bounds is off by less than 1e-3 pixel
// (and a rounded pixel centre by less than 1e-4), so widening each bound by
// 0.01 pixel keeps every pixel whose centre passes the bbox test.
__device__ __forceinline__ void pix_range(float vmin, float vmax, int size, int& lo, int& hi) {
    float a = ((float)size * (1.0f - vmax) - 1.0f) * 0.5f;
    float b = ((float)size * (1.0f - vmin) - 1.0f) * 0.5f;
    a = fminf(fmaxf(a, -2.0f), (float)size + 1.0f);
    b = fminf(fmaxf(b, -2.0f), (float)size + 1.0f);
    lo = (int)ceilf(a - 0.01f);
    hi = (int)floorf(b + 0.01f);
    if (lo < 0) lo = 0;
    if (hi > size - 1) hi = size - 1;
}

// Bins [bx0, bx1] x [by0, by1] (bin_size bs) whose pixels may count a face
// with grown box bb; false when the face counts nowhere on the H x W image
// (a face that never counts has an empty box).  The binning pass and the
// backward use this same function, so they agree on every face's bins.
__device__ __forceinline__ bool face_bins_of_box(const float4 bb, int H, int W, int bs, int& bx0, int& bx1, int& by0,
                                                 int& by1) {
    int c0, c1, r0, r1;
    pix_range(bb.x, bb.y, W, c0, c1);
    pix_range(bb.z, bb.w, H, r0, r1);
    if (c1 < c0 || r1 < r0) return false;
    bx0 = c0 / bs;
    bx1 = c1 / bs;
    by0 = r0 / bs;
    by1 = r1 / bs;
    return true;
}
__device__ __forceinline__ bool face_bins(const FaceRec& R, int H, int W, int bs, int& bx0, int& bx1, int& by0,
                                          int& by1) {
    if (!R.ok()) return false;
    return face_bins_of_box(R.bb, H, W, bs, bx0, bx1, by0, by1);
}

// Sort key: ascending z, then ascending face id, as one unsigned 64-bit
// integer (the bit pattern of a non-negative float is monotone in its value).
// Only z >= 0 is ever keyed (-0 becomes +0), so a key's top bit is clear and
// its top twelve bits are at most those of +inf as a float; read as an IEEE
// double the key is therefore a non-negative number below +inf (a subnormal
// when z = 0), and doubles of that range order exactly as their bit patterns.
// The empty key is +inf as a double, above every real key.
__device__ __forceinline__ uint64_t make_key(float z, int fid) {
    uint32_t zb = (z == 0.0f) ? 0u : __float_as_uint(z);
    return ((uint64_t)zb << 32) | (uint32_t)fid;
}
constexpr uint64_t kEmptyKey = 0x7ff0000000000000ull;

__device__ __forceinline__ double key_as_f64(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint64_t f64_as_key(double d) { return (uint64_t)__double_as_longlong(d); }

// Compare-exchange: a <- min, b <- max, as one FP64 min and one FP64 max
// (two instructions, against a 64-bit compare and four selects).  Both are
// exact on the keys' range: no NaN ever occurs, and the kernels keep FP64
// subnormals (denormal mode "preserve"), so the keys of z = 0 stay distinct.
__device__ __forceinline__ void cex(uint64_t& a, uint64_t& b) {
    const double x = key_as_f64(a), y = key_as_f64(b);
    a = f64_as_key(__builtin_fmin(x, y));
    b = f64_as_key(__builtin_fmax(x, y));
}
__device__ __forceinline__ uint64_t key_min(uint64_t a, uint64_t b) {
    return f64_as_key(__builtin_fmin(key_as_f64(a), key_as_f64(b)));
}

// Sorts eight keys ascending with a 19-comparator network.
__device__ __forceinline__ void sort8(uint64_t (&b)[8]) {
    cex(b[0], b[2]); cex(b[1], b[3]); cex(b[4], b[6]); cex(b[5], b[7]);
    cex(b[0], b[4]); cex(b[1], b[5]); cex(b[2], b[6]); cex(b[3], b[7]);
    cex(b[0], b[1]); cex(b[2], b[3]); cex(b[4], b[5]); cex(b[6], b[7]);
    cex(b[2], b[4]); cex(b[3], b[5]);
    cex(b[1], b[4]); cex(b[3], b[6]);
    cex(b[1], b[2]); cex(b[3], b[4]); cex(b[5], b[6]);
}

constexpr bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Register-resident sorted list of the KB smallest keys, only ever indexed
// with compile-time constants.
template <int KB>
struct TopK {
    uint64_t q[KB];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int i = 0; i < KB; ++i) q[i] = kEmptyKey;
    }
    // Keeps the KB smallest of the queue and eight new keys (absent keys are
    // kEmptyKey).  The batch is sorted, then one half-cleaner step
    // q[i] = min(q[i], b[KB-1-i]) leaves the KB smallest of both as a bitonic
    // sequence, and a bitonic merge sorts it: about four compare-exchanges
    // per key for KB = 16, against KB for one insertion at a time.
    __device__ __forceinline__ void merge8(uint64_t (&b)[8]) {
        sort8(b);
        constexpr int M = KB < 8 ? KB : 8;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int qi = KB - M + i;
            q[qi] = key_min(b[M - 1 - i], q[qi]);
        }
#pragma unroll
        for (int d = KB / 2; d >= 1; d /= 2) {
#pragma unroll
            for (int i = 0; i < KB; ++i)
                if (!(i & d)) cex(q[i], q[i + d]);
        }
    }
    // merge8 confined to the first S slots, for a lane whose queue holds c
    // keys and gets n new ones with c + n <= S: the slots from S on stay
    // empty, the eight keys the half-cleaner drops are empty ones, and the
    // merge costs log2(S) stages of S / 2 compare-exchanges instead of
    // log2(KB) stages of KB / 2.
    template <int S>
    __device__ __forceinline__ void merge8_prefix(uint64_t (&b)[8]) {
        static_assert(S >= 8 && S <= KB && is_pow2(S), "prefix size");
        sort8(b);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int qi = S - 8 + i;
            q[qi] = key_min(b[7 - i], q[qi]);
        }
#pragma unroll
        for (int d = S / 2; d >= 1; d /= 2) {
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (!(i & d)) cex(q[i], q[i + d]);
        }
    }
    // Adds eight keys: batched merge for power-of-two queues, else one at a time.
    __device__ __forceinline__ void push8(uint64_t (&b)[8]) {
        if constexpr (is_pow2(KB)) {
            merge8(b);
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) insert(b[u]);
        }
    }
    // Branch-free insertion: every slot is a compare-exchange with the
    // travelling key, so the array is only indexed with compile-time
    // constants; `want` masks lanes with nothing to insert.
    __device__ __forceinline__ void insert(uint64_t key, bool want = true) {
        if (!want) key = kEmptyKey;
#pragma unroll
        for (int i = 0; i < KB; ++i) cex(q[i], key);
    }
};

// Work item of workgroup L of a T-workgroup grid, such that every XCD works
// through one contiguous range of the items.  The hardware hands workgroups
// to the chip's kXcds XCDs in turn (L to XCD L mod kXcds, the (L / kXcds)-th
// there); each XCD has its own L2, so neighbouring items, which share their
// input (a tile's faces are mostly its neighbours' faces too), hit in one L2
// instead of being spread over all of them.  A bijection of [0, T): XCD x
// takes items [x q + min(x, r), (x + 1) q + min(x + 1, r)) with q = T / kXcds,
// r = T mod kXcds.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t L, int64_t T) {
    const int64_t q = T / kXcds, r = T - q * kXcds;
    const int64_t x = L % kXcds, k = L / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Largest value of v over the wave.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// element e of a pass that stages `per` values per pixel: pixel e / per
__device__ __forceinline__ int stage_pixel(int e, float inv_per) { return (int)(((float)e + 0.5f) * inv_per); }

// Pixels of the 8x8 tile (x0, y0) whose centres the box [bb.x, bb.y] x
// [bb.z, bb.w] may contain, from the same conservative pixel ranges as the
// binning (an empty box gives 0).
__device__ __forceinline__ uint64_t tile_mask(const float4 bb, int H, int W, int x0, int y0, float tx_lo, float tx_hi,
                                              float ty_lo, float ty_hi) {
    // most faces of a single-pass tile miss it: reject those on the box alone
    if (bb.y < tx_lo || bb.x > tx_hi || bb.w < ty_lo || bb.z > ty_hi) return 0ull;
    int c0, c1, r0, r1;
    pix_range(bb.x, bb.y, W, c0, c1);
    pix_range(bb.z, bb.w, H, r0, r1);
    c0 = max(c0 - x0, 0);
    c1 = min(c1 - x0, kTile - 1);
    r0 = max(r0 - y0, 0);
    r1 = min(r1 - y0, kTile - 1);
    if (c1 < c0 || r1 < r0) return 0ull;
    const uint64_t cols = (uint64_t)((0xffu >> (kTile - 1 - (c1 - c0))) << c0) * 0x0101010101010101ull;
    const uint64_t rows = (~0ull >> (8 * (kTile - 1 - r1))) & (~0ull << (8 * r0));
    return cols & rows;
}

// Pixels of the 8x8 tile (x0, y0) that a face may count for, by its three
// edge lines: a pixel counts only inside the triangle or within sqrt(blur)
// of it, and the triangle lies on the inner side of each edge line, so a
// pixel more than rg = sqrt(blur) (1 + 1e-4) + 1e-6 outside any one line
// cannot count (rg is the box pad's radius: it covers the FP32 error of the
// distance test).  Per line i the edge function at pixel (r, c) of the tile
// is e_i(r, c) = e_i(0, 0) - c (2/W) A_i - r (2/H) B_i (A_i, B_i its x and y
// coefficients), and the kept columns of row r are those with
// sgn(E) e_i > -rg |edge_i|, a half-line in c.  e_i(0, 0), the thresholds
// the row terms and the column bounds are FP64 (their rounding is far below
// the margin rg leaves over the test's own error); only the clamped bound is
// converted.  Conservative: every pixel the test accepts is kept.
struct EdgeGeo {
    double2 pa, ab, ac;
    double E;
};
__device__ __forceinline__ double2 f4_as_d2(const float4 v) {
    return make_double2(__hiloint2double(__float_as_int(v.y), __float_as_int(v.x)),
                        __hiloint2double(__float_as_int(v.w), __float_as_int(v.z)));
}
template <class Rec>
__device__ __forceinline__ uint64_t edge_mask(const Rec& R, double rg, int H, int W, int x0, int y0) {
    const double px = 1.0 - (double)(2 * x0 + 1) / (double)W, py = 1.0 - (double)(2 * y0 + 1) / (double)H;
    const double dx = px - R.pa.x, dy = py - R.pa.y;
    const double sg = R.E > 0.0 ? 1.0 : -1.0;
    // e1 = cross(p - a, c - a), e2 = cross(b - a, p - a), e0 = E - e1 - e2
    const double e1 = dx * R.ac.y - dy * R.ac.x;
    const double e2 = R.ab.x * dy - R.ab.y * dx;
    const double e0 = (R.E - e1) - e2;
    const double A1 = R.ac.y, B1 = -R.ac.x, A2 = -R.ab.y, B2 = R.ab.x;
    const double A0 = -(A1 + A2), B0 = -(B1 + B2);
    // edge lengths: e0 <-> (b, c), e1 <-> (c, a), e2 <-> (a, b)
    const double bcx = R.ac.x - R.ab.x, bcy = R.ac.y - R.ab.y;
    const double l0 = sqrt(bcx * bcx + bcy * bcy), l1 = sqrt(R.ac.x * R.ac.x + R.ac.y * R.ac.y),
                 l2 = sqrt(R.ab.x * R.ab.x + R.ab.y * R.ab.y);
    const double sx = 2.0 / (double)W, sy = 2.0 / (double)H;
    // keep (r, c) iff c * g_i < k_i - r * h_i for all i, with
    //   g_i = sg sx A_i,  k_i = sg e_i(0,0) + rg l_i,  h_i = sg sy B_i
    const double g[3] = {sg * sx * A0, sg * sx * A1, sg * sx * A2};
    const double k[3] = {sg * e0 + rg * l0, sg * e1 + rg * l1, sg * e2 + rg * l2};
    const double h[3] = {sg * sy * B0, sg * sy * B1, sg * sy * B2};
    double ig[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ig[i] = g[i] != 0.0 ? 1.0 / g[i] : 0.0;
    uint64_t m = 0ull;
#pragma unroll
    for (int r = 0; r < kTile; ++r) {
        float lo = 0.0f, hi = (float)(kTile - 1);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double kr = k[i] - (double)r * h[i];
            if (g[i] == 0.0) {
                if (!(kr > 0.0)) hi = -1.0f;  // the whole row is outside this line
            } else {
                // the row's bound on c, clamped to [-2, 9] before the conversion
                const float b = (float)fmin(fmax(kr * ig[i], -2.0), 9.0);
                if (g[i] > 0.0)
                    hi = fminf(hi, floorf(b));  // c <= k / g (c = k / g kept: conservative)
                else
                    lo = fmaxf(lo, ceilf(b));
            }
        }
        if (lo <= hi) {
            const int a = (int)lo, z = (int)hi;
            const uint32_t row = (0xffu >> (kTile - 1 - z)) & (0xffu << a);
            m |= (uint64_t)row << (8 * r);
        }
    }
    return m;
}

// One global atomic per distinct bucket of a wave (tiles of a wave mostly
// share a few buckets): returns the wave's base position in
// that bucket for the calling lane, whose rank among the wave's tiles of the
// bucket is added.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_bucket_slot(int* __restrict__ hist, int bucket) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t active = __ballot(bucket >= 0);
    int pos = -1;
    while (active) {  // uniform: active is the same on every lane
        const int leader = __ffsll((unsigned long long)active) - 1;
        const int bl = __shfl(bucket, leader);
        const uint64_t same = __ballot(bucket == bl);
        int base = 0;
        if (lane == leader) base = atomicAdd(&hist[bl], __popcll(same));
        base = __shfl(base, leader);
        if (bucket == bl) pos = base + __popcll(same & below);
        active &= ~same;
    }
    return pos;
}

}  // namespace rast
