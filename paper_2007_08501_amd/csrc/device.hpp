// device.hpp -- per-face and per-pixel arithmetic of the rasterizer, FP32, gfx950.
//
// Everything that decides whether a face counts for a pixel, and the values
// written for it, lives here so that the single-pass and the binned forward
// and the backward evaluate every (pixel, face) pair with the same
// instructions (the library is built with -ffp-contract=off, so the compiler
// cannot fuse differently in different kernels).
//
// Accuracy.  Faces seen edge-on (near a silhouette) project to slivers whose
// doubled area E is tiny, and a barycentric w_i = e_i / E amplifies any error
// of the edge function e_i by 1/E.  FP32 rounding of a pixel-to-vertex offset
// or of an edge vector is then far above the 1e-5 target, so both are carried
// exactly as unevaluated sums hi + lo (Knuth's two-sum), the edge functions
// are formed as Kahan FMA differences of products of the hi parts plus
// first-order corrections from the lo parts, and the third barycentric comes
// from E - e1 - e2.  Each w_i is then accurate to a few units in the last
// place of max(1, abs(w_i)), whatever the shape of the face.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rast {

constexpr float kEpsArea = 1e-8f;  // faces with abs(2 * signed area) below this never count
constexpr int kTile = 8;           // forward work unit: 8x8 pixels = one wave64

// Workspace header (int32 words); the header occupies the first 256 bytes.
enum : int {
    kHdrStatus = 0,     // sticky status bits (kStatOverflow | kStatMesh)
    kHdrMaxCount = 1,   // largest bin count seen
    kHdrWorkNext = 2,   // persistent scheduler: next work item
    kHdrWorkTotal = 3,  // persistent scheduler: number of work items
    kHdrBigCount = 8,   // backward: number of faces with large pixel boxes
    kHdrBigNext = 9,    // backward: next large face to scan
    kHdrWords = 64,
};
enum : int { kStatOverflow = 1, kStatMesh = 2 };

// x = hi + lo exactly, hi = fl(a - b) (Knuth's two-sum applied to a + (-b)).
__device__ __forceinline__ void two_diff(float a, float b, float& hi, float& lo) {
    float s = a - b;
    float bb = s - a;
    lo = (a - (s - bb)) - (b + bb);
    hi = s;
}

// Pixel centre in NDC as an unevaluated sum hi + lo:
// x = 1 - (2c+1)/W, y = 1 - (2r+1)/H.  lo is 0 for power-of-two sizes.
__device__ __forceinline__ void pix_center(int c, int W, float& hi, float& lo) {
    float num = (float)(2 * c + 1);
    float q = num / (float)W;                // correctly rounded quotient
    float rem = fmaf(-q, (float)W, num);     // exact remainder num - q*W
    float h, l;
    two_diff(1.0f, q, h, l);
    hi = h;
    lo = l - rem / (float)W;
}
// Rounded pixel centre (equal to hi above); used for tile extents and culls.
__device__ __forceinline__ float pix_x(int c, int W) { return 1.0f - (float)(2 * c + 1) / (float)W; }
__device__ __forceinline__ float pix_y(int r, int H) { return 1.0f - (float)(2 * r + 1) / (float)H; }

struct Pix {
    float x, y, xl, yl;  // centre hi parts and lo parts
};
__device__ __forceinline__ Pix make_pix(int r, int c, int H, int W) {
    Pix p;
    pix_center(c, W, p.x, p.xl);
    pix_center(r, H, p.y, p.yl);
    return p;
}

// a*b - c*d with one rounding error's worth of accuracy (Kahan's FMA
// difference of products).
__device__ __forceinline__ float dop(float a, float b, float c, float d) {
    float w = c * d;
    float e = fmaf(-c, d, w);
    float f = fmaf(a, b, -w);
    return f + e;
}

// Per-face record, 80 bytes, built once per call by the setup kernel.
//   q0  ax, ay, E, 1/E                 (E = doubled signed area = cross(b-a, c-a))
//   q1  (b-a).x, (b-a).y, (c-a).x, (c-a).y    rounded edge vectors
//   q2  their rounding residuals (exact: edge = q1 + q2)
//   q3  az, bz - az, cz - az, mesh id (int bits; -1 = never counts)
//   q4  xmin, xmax, ymin, ymax: xy bbox grown by sqrt(blur) plus a pad;
//       empty (+inf, -inf) for faces that never count
struct FaceRec {
    float4 q0, q1, q2, q3, q4;
    __device__ __forceinline__ int mesh() const { return __float_as_int(q3.w); }
    __device__ __forceinline__ bool ok() const { return __float_as_int(q3.w) >= 0; }
    __device__ __forceinline__ float invE() const { return q0.w; }
};

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// cross(u, v) for u = uh + ul, v = vh + vl: Kahan product of the hi parts
// plus the first-order terms of the residuals (the lo*lo term is below the
// rounding of the result).
__device__ __forceinline__ float cross_acc(float uhx, float uhy, float ulx, float uly, float vhx, float vhy, float vlx,
                                           float vly) {
    float main = dop(uhx, vhy, uhy, vhx);
    float corr = fmaf(uhx, vly, fmaf(ulx, vhy, -fmaf(uhy, vlx, uly * vhx)));
    return main + corr;
}

// Builds the record of face (a, b, c).  rb = sqrt(blur_radius) in NDC units.
__device__ __forceinline__ FaceRec make_rec(float ax, float ay, float az, float bx, float by, float bz, float cx,
                                            float cy, float cz, float rb, int mesh) {
    FaceRec R;
    float abx, abxl, aby, abyl, acx, acxl, acy, acyl;
    two_diff(bx, ax, abx, abxl);
    two_diff(by, ay, aby, abyl);
    two_diff(cx, ax, acx, acxl);
    two_diff(cy, ay, acy, acyl);
    float E = cross_acc(abx, aby, abxl, abyl, acx, acy, acxl, acyl);
    bool ok = mesh >= 0 && fabsf(E) >= kEpsArea && finite3(ax, ay, az) && finite3(bx, by, bz) &&
              finite3(cx, cy, cz);
    R.q0 = make_float4(ax, ay, E, ok ? 1.0f / E : 0.0f);
    R.q1 = make_float4(abx, aby, acx, acy);
    R.q2 = make_float4(abxl, abyl, acxl, acyl);
    R.q3 = make_float4(az, bz - az, cz - az, __int_as_float(ok ? mesh : -1));
    if (ok) {
        // The pad covers the FP32 error of the distance test: a pixel whose
        // FP32 squared distance is < blur is never farther than rb*(1+1e-6)+1e-7.
        float pad = rb * 1e-4f + 1e-6f;
        float g = rb + pad;
        R.q4 = make_float4(fminf(ax, fminf(bx, cx)) - g, fmaxf(ax, fmaxf(bx, cx)) + g,
                           fminf(ay, fminf(by, cy)) - g, fmaxf(ay, fmaxf(by, cy)) + g);
    } else {
        R.q4 = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    }
    return R;
}

// Squared distance from the origin (the pixel) to segment S + t*V, t in [0,1],
// with S, V in pixel-relative coordinates; returns the clamped parameter too.
__device__ __forceinline__ float seg_d2(float sx, float sy, float vx, float vy, float& u) {
    float l2 = vx * vx + vy * vy;
    float t = -(sx * vx + sy * vy);
    float uu = 0.0f;
    if (l2 > 0.0f) {
        uu = t * __builtin_amdgcn_rcpf(l2);
        uu = uu < 0.0f ? 0.0f : (uu > 1.0f ? 1.0f : uu);
    }
    u = uu;
    float qx = fmaf(uu, vx, sx), qy = fmaf(uu, vy, sy);
    return qx * qx + qy * qy;
}

// Everything the forward writes for one (pixel, face) pair, and what the
// backward needs besides.
struct Eval {
    float w0, w1, w2;  // barycentrics
    float z;
    float d2;     // squared distance to the nearest boundary point
    float u;      // parameter of the nearest point on the nearest edge
    int edge;     // nearest edge: 0 = (a,b), 1 = (b,c), 2 = (c,a); lowest index on ties
    bool inside;  // all three barycentrics > 0
    float sx, sy; // p - a (rounded): the pixel relative to vertex a
};

// Barycentrics, z and inside-ness of pixel p in face R.
__device__ __forceinline__ void eval_bary(const FaceRec& R, const Pix& p, float& w0, float& w1, float& w2, float& z,
                                          bool& inside, float& sx, float& sy) {
    // s = p - a exactly as sh + sl
    float shx, slx, shy, sly;
    two_diff(p.x, R.q0.x, shx, slx);
    two_diff(p.y, R.q0.y, shy, sly);
    slx += p.xl;
    sly += p.yl;
    // e1 = cross(p - a, c - a), e2 = cross(b - a, p - a), e0 = E - e1 - e2
    float e1 = cross_acc(shx, shy, slx, sly, R.q1.z, R.q1.w, R.q2.z, R.q2.w);
    float e2 = cross_acc(R.q1.x, R.q1.y, R.q2.x, R.q2.y, shx, shy, slx, sly);
    float e0 = (R.q0.z - e1) - e2;
    float invE = R.q0.w;
    w0 = e0 * invE;
    w1 = e1 * invE;
    w2 = e2 * invE;
    // z = w0 az + w1 bz + w2 cz, rearranged with w0 = 1 - w1 - w2 so that the
    // large common depth az is added last
    z = fmaf(w2, R.q3.z, w1 * R.q3.y) + R.q3.x;
    inside = (w0 > 0.0f) && (w1 > 0.0f) && (w2 > 0.0f);
    sx = shx;
    sy = shy;
}

// Squared distance to the triangle boundary and its nearest edge, from the
// pixel offset s = p - a.
__device__ __forceinline__ float eval_dist(const FaceRec& R, float sx, float sy, int& edge, float& u) {
    float Ax = -sx, Ay = -sy;                         // a - p
    float Bx = Ax + R.q1.x, By = Ay + R.q1.y;         // b - p
    float u0, u1, u2;
    float d0 = seg_d2(Ax, Ay, R.q1.x, R.q1.y, u0);
    float d1 = seg_d2(Bx, By, R.q1.z - R.q1.x, R.q1.w - R.q1.y, u1);
    float d2 = seg_d2(Ax + R.q1.z, Ay + R.q1.w, -R.q1.z, -R.q1.w, u2);
    float d = d0;
    int e = 0;
    float uu = u0;
    if (d1 < d) { d = d1; e = 1; uu = u1; }
    if (d2 < d) { d = d2; e = 2; uu = u2; }
    edge = e;
    u = uu;
    return d;
}

__device__ __forceinline__ void eval_full(const FaceRec& R, const Pix& p, Eval& o) {
    eval_bary(R, p, o.w0, o.w1, o.w2, o.z, o.inside, o.sx, o.sy);
    o.d2 = eval_dist(R, o.sx, o.sy, o.edge, o.u);
}

__device__ __forceinline__ bool in_bbox(const FaceRec& R, const Pix& p) {
    return p.x >= R.q4.x && p.x <= R.q4.y && p.y >= R.q4.z && p.y <= R.q4.w;
}

// Does face R count for pixel p?  On success z is its depth.
__device__ __forceinline__ bool face_counts(const FaceRec& R, const Pix& p, float blur, float& z) {
    if (!in_bbox(R, p)) return false;
    float w0, w1, w2, sx, sy;
    bool inside;
    eval_bary(R, p, w0, w1, w2, z, inside, sx, sy);
    if (!(z >= 0.0f)) return false;
    if (inside) return true;
    int e;
    float u;
    float d2 = eval_dist(R, sx, sy, e, u);
    return d2 < blur;
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

// Bins [bx0, bx1] x [by0, by1] (bin_size bs) whose pixels may count face R;
// false when the face counts nowhere on the H x W image.  The binning pass
// and the backward use this same function, so they agree on every face's
// bins.
__device__ __forceinline__ bool face_bins(const FaceRec& R, int H, int W, int bs, int& bx0, int& bx1, int& by0,
                                          int& by1) {
    if (!R.ok()) return false;
    int c0, c1, r0, r1;
    pix_range(R.q4.x, R.q4.y, W, c0, c1);
    pix_range(R.q4.z, R.q4.w, H, r0, r1);
    if (c1 < c0 || r1 < r0) return false;
    bx0 = c0 / bs;
    bx1 = c1 / bs;
    by0 = r0 / bs;
    by1 = r1 / bs;
    return true;
}

// Sort key: ascending z, then ascending face id, as one unsigned 64-bit
// integer (the bit pattern of a non-negative float is monotone in its value).
__device__ __forceinline__ uint64_t make_key(float z, int fid) {
    uint32_t zb = (z == 0.0f) ? 0u : __float_as_uint(z);
    return ((uint64_t)zb << 32) | (uint32_t)fid;
}
constexpr uint64_t kEmptyKey = ~0ull;

// Register-resident sorted list of the KB smallest keys; every slot is a
// compare-exchange with the travelling key, so the array is only ever
// indexed with compile-time constants.
template <int KB>
struct TopK {
    uint64_t q[KB];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int i = 0; i < KB; ++i) q[i] = kEmptyKey;
    }
    __device__ __forceinline__ void insert(uint64_t key) {
        if (key >= q[KB - 1]) return;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            uint64_t lo = key < q[i] ? key : q[i];
            uint64_t hi = key < q[i] ? q[i] : key;
            q[i] = lo;
            key = hi;
        }
    }
};

}  // namespace rast
