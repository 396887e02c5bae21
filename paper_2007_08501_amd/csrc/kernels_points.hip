// kernels_points.hip -- point-cloud rasterizer and compositing for gfx950.
//
//   pt_count      one thread per point: cloud id, home tile, rank in that tile
//   pt_scan_*     exclusive scan of the per-tile counts into tile starts
//   pt_scatter    one thread per point: 16-byte record at its sorted slot
//   pt_raster     one wave per 8x8 tile: candidates from the home lists of
//                 the tiles that can reach it, cull, exact FP64 test per
//                 pixel, K nearest along z in registers, write the fragments
//   pt_bwd        one thread per sorted point: gathers the gradient of its
//                 own slots from the pixels its disc covers (no atomics)
//   composite     one thread per pixel: Alpha / Norm compositing, backward
//
// Paper, Section 3.3: every point is splatted to a disc of radius r in screen
// space; each pixel keeps the K points nearest along z whose discs cover it,
// with their depth and squared xy distance to the pixel centre, and the
// features of those points are blended by Alpha compositing or by a
// normalised weighted sum.  The rasterizer follows the mesh rasterizer's
// scheme (tiles first, then pixels, register top-K per pixel); the coarse
// pass is a counting sort of the points by home tile instead of per-bin
// lists, so it has no capacity limit.
#include "device.hpp"
#include "launch.hpp"

namespace rast {

// Home tile of a point: the tile holding the first pixel (lowest row, lowest
// column) of the pixel ranges its disc may cover.  A disc then reaches at
// most rx tiles to the right of and ry tiles below its home tile, so a tile
// collects its candidates from the home lists of the tiles at most rx to its
// left and ry above it.
__device__ __forceinline__ bool disc_pixels(float x, float y, float r, int H, int W, int& c0, int& c1, int& r0,
                                            int& r1) {
    pix_range(x - r, x + r, W, c0, c1);
    pix_range(y - r, y + r, H, r0, r1);
    return c0 <= c1 && r0 <= r1;
}

struct PtArgs {
    const float* pts;       // (P,3)
    const int64_t* first;   // (N) cloud ranges
    const int64_t* np;
    int64_t P;
    int N, H, W, K;
    float r;                // radius
    double r2;              // radius^2, FP64
    int tiles_x, tiles_y, rx, ry;
    int64_t T;              // tiles in the batch
    int* hdr;
    int* start;             // T+1: counts, then tile starts
    int* bsum;              // scan block sums
    int* home;              // (P) home tile or -1
    int* rank;              // (P) rank within the home tile
    float4* sorted;         // (P) x, y, z, id
    int32_t* idx;           // (N,H,W,K) outputs
    float* zbuf;
    float* dists;
};

__global__ __launch_bounds__(256) void pt_count_kernel(PtArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.N) {
        // cloud range check: inside [0, P] and ascending without overlap
        const int64_t f = a.first[p], c = a.np[p];
        bool bad = f < 0 || c < 0 || f + c > a.P;
        if (p > 0) bad = bad || f < a.first[p - 1] + a.np[p - 1];
        if (bad) atomicOr(&a.hdr[kHdrStatus], kStatMesh);
    }
    if (p >= a.P) return;
    const int n = find_mesh(a.first, a.np, a.N, p);
    const float x = a.pts[3 * p], y = a.pts[3 * p + 1], z = a.pts[3 * p + 2];
    int h = -1, rk = 0, c0, c1, r0, r1;
    // points behind the camera or covering no pixel take no part
    if (n >= 0 && z >= 0.0f && disc_pixels(x, y, a.r, a.H, a.W, c0, c1, r0, r1)) {
        h = (int)(((int64_t)n * a.tiles_y + r0 / kTile) * a.tiles_x + c0 / kTile);
        rk = atomicAdd(&a.start[h], 1);
    }
    a.home[p] = h;
    a.rank[p] = rk;
}

// Exclusive scan of start[0, T) in place, start[T] = total, in three passes:
// block sums, a scan of the block sums, then each block's scan plus its
// offset.  A block covers kScanTile counts, four per thread.
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4 * kScanThreads;

// Exclusive prefix of v over the block and the block's total.
__device__ __forceinline__ int block_exclusive(int v, int* sm, int& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sm[w] = incl;
    __syncthreads();
    if (threadIdx.x < 64) {
        int s = lane < kScanThreads / 64 ? sm[lane] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(s, o);
            if (lane >= o) s += t;
        }
        if (lane < kScanThreads / 64) sm[lane] = s;
    }
    __syncthreads();
    const int base = w > 0 ? sm[w - 1] : 0;
    total = sm[kScanThreads / 64 - 1];
    __syncthreads();
    return base + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void pt_scan_sums_kernel(const int* __restrict__ c, int64_t T,
                                                                    int* __restrict__ bsum) {
    __shared__ int sm[kScanThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    int v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) v += (i0 + j < T) ? c[i0 + j] : 0;
    int total;
    block_exclusive(v, sm, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// one block: exclusive scan of the nb block sums in place, bsum[nb] = total
__global__ __launch_bounds__(kScanThreads) void pt_scan_top_kernel(int* __restrict__ bsum, int64_t nb) {
    __shared__ int sm[kScanThreads / 64];
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t i = b0 + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_exclusive(v, sm, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void pt_scan_apply_kernel(int* __restrict__ c, int64_t T,
                                                                     const int* __restrict__ bsum, int64_t nb) {
    __shared__ int sm[kScanThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    int v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = (i0 + j < T) ? c[i0 + j] : 0;
        s += v[j];
    }
    int total;
    int ex = bsum[blockIdx.x] + block_exclusive(s, sm, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (i0 + j < T) c[i0 + j] = ex;
        ex += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c[T] = bsum[nb];
}

__global__ __launch_bounds__(256) void pt_scatter_kernel(PtArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const int h = a.home[p];
    if (h < 0) return;
    const float x = a.pts[3 * p], y = a.pts[3 * p + 1], z = a.pts[3 * p + 2];
    a.sorted[a.start[h] + a.rank[p]] = make_float4(x, y, z, __int_as_float((int)p));
}

// ---------------------------------------------------------------------------
// Fine pass.  Candidates are gathered a wave-wide chunk at a time, culled on
// their pixel ranges and compacted into an LDS batch of up to kPtBatch
// points; a full batch is then tested per pixel in FP64 (the squared
// distance in the same operations and order as a plain evaluation, so the
// decision is reproducible bit for bit), each lane lists its hits, and the
// lists go through the register top-K eight keys at a time.
// ---------------------------------------------------------------------------
constexpr int kPtBatch = 128;
static_assert(kPtBatch <= 256, "per-lane lists hold byte indices");

struct PtLds {
    double2 xy[kPtBatch];
    uint64_t key[kPtBatch];                 // (z, id) sort key
    unsigned char lst[kPtBatch * 64];       // entry i of lane l at [i * 64 + l]
};

__device__ __forceinline__ double pt_d2(double x, double y, double px, double py) {
    const double dx = x - px, dy = y - py;
    return dx * dx + dy * dy;
}

template <int KB>
__device__ __forceinline__ void pt_batch(const PtArgs& a, PtLds& L, TopK<KB>& top, int m, bool live, double px,
                                         double py) {
    __syncthreads();
    const int lane = threadIdx.x & 63;
    unsigned char* my = L.lst + lane;
    int nl = 0;
    for (int j = 0; j < m; ++j) {
        const double2 q = L.xy[j];
        if (live && pt_d2(q.x, q.y, px, py) < a.r2) my[64 * nl++] = (unsigned char)j;
    }
    const int nmax = wave_max(nl);
    for (int i0 = 0; i0 < nmax; i0 += 8) {
        uint64_t b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = (i0 + u < nl) ? L.key[my[64 * (i0 + u)]] : kEmptyKey;
        top.push8(b);
    }
    __syncthreads();
}

// Stores slots [g0, g0 + gw) of the tile's pixels from an LDS stage (pixel
// major, stride G + 1) so that consecutive lanes write consecutive words.
template <int G, bool V4, bool EXACT>
__device__ __forceinline__ void pt_store(uint32_t* __restrict__ out, const uint32_t* st, int K, int rowK, int g0,
                                         int gw, int rows, int cols) {
    constexpr int S = G + 1;
    const int lane = threadIdx.x & 63;
    if constexpr (V4) {
        constexpr int Q = G / 4;
#pragma unroll
        for (int e0 = 0; e0 < 64 * Q; e0 += 64) {
            const int e = e0 + lane;
            const int px = e / Q, q = e - px * Q;
            const int r = px >> 3, c = px & 7;
            if (r < rows && c < cols) {
                const uint32_t* si = st + px * S + 4 * q;
                *reinterpret_cast<uint4*>(out + r * rowK + c * K + g0 + 4 * q) = make_uint4(si[0], si[1], si[2], si[3]);
            }
        }
    } else {
        const float inv = 1.0f / (float)gw;
#pragma unroll
        for (int e0 = 0; e0 < 64 * G; e0 += 64) {
            const int e = e0 + lane;
            if (e >= 64 * gw) break;
            const int px = EXACT ? e / gw : stage_pixel(e, inv);
            const int k = e - px * gw;
            const int r = px >> 3, c = px & 7;
            if (r < rows && c < cols) out[r * rowK + c * K + g0 + k] = st[px * S + k];
        }
    }
}

template <int KB, bool EXACT>
__device__ __forceinline__ void pt_write(const PtArgs& a, PtLds& L, const TopK<KB>& top, double px, double py, int n,
                                         int tx, int ty) {
    const int lane = threadIdx.x & 63;
    const int K = EXACT ? KB : a.K;
    const int rows = min(kTile, a.H - ty * kTile), cols = min(kTile, a.W - tx * kTile);
    const int64_t pix0 = ((int64_t)n * a.H + ty * kTile) * a.W + tx * kTile;
    const int rowK = a.W * K;
    constexpr bool V4 = EXACT && (KB % 4 == 0);
    constexpr int G = KB < 16 ? KB : 16;
    constexpr int S = G + 1;
    static_assert(sizeof(PtLds) >= sizeof(uint32_t) * 64 * S * 2, "staging exceeds the tile LDS");
    uint32_t* const idx_t = reinterpret_cast<uint32_t*>(a.idx + pix0 * K);
    uint32_t* const z_t = reinterpret_cast<uint32_t*>(a.zbuf + pix0 * K);
    uint32_t* const d_t = reinterpret_cast<uint32_t*>(a.dists + pix0 * K);
    uint32_t* sid = reinterpret_cast<uint32_t*>(&L);
    uint32_t* sz = sid + 64 * S;
    const uint32_t neg1 = __float_as_uint(-1.0f);
#pragma unroll
    for (int g0 = 0; g0 < KB; g0 += G) {
        if (g0 >= K) continue;  // K is uniform: the whole wave skips
        const int gw = EXACT ? G : min(G, K - g0);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const uint64_t key = top.q[g0 + k];
            const bool empty = key == kEmptyKey;
            sid[lane * S + k] = empty ? 0xffffffffu : (uint32_t)key;
            sz[lane * S + k] = empty ? neg1 : (uint32_t)(key >> 32);
        }
        __syncthreads();
        pt_store<G, V4, EXACT>(idx_t, sid, K, rowK, g0, gw, rows, cols);
        pt_store<G, V4, EXACT>(z_t, sz, K, rowK, g0, gw, rows, cols);
        __syncthreads();
        // squared distances, recomputed in FP64 exactly as the test did
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const uint64_t key = top.q[g0 + k];
            float d = -1.0f;
            if (key != kEmptyKey) {
                const int64_t id = (int64_t)(uint32_t)key;
                d = (float)pt_d2((double)a.pts[3 * id], (double)a.pts[3 * id + 1], px, py);
            }
            sid[lane * S + k] = __float_as_uint(d);
        }
        __syncthreads();
        pt_store<G, V4, EXACT>(d_t, sid, K, rowK, g0, gw, rows, cols);
        __syncthreads();
    }
}

template <int KB, bool EXACT>
__global__ __launch_bounds__(64) void pt_raster_kernel(PtArgs a) {
    __shared__ PtLds L;
    const int tx = blockIdx.x, ty = blockIdx.y, n = blockIdx.z;
    const int lane = threadIdx.x & 63;
    const int r = ty * kTile + (lane >> 3), c = tx * kTile + (lane & 7);
    const bool live = r < a.H && c < a.W;
    const double px = 1.0 - (double)(2 * c + 1) / (double)a.W;
    const double py = 1.0 - (double)(2 * r + 1) / (double)a.H;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int x1 = min(x0 + kTile, a.W) - 1, y1 = min(y0 + kTile, a.H) - 1;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    TopK<KB> top;
    top.init();
    int m = 0;
    for (int yy = max(ty - a.ry, 0); yy <= ty; ++yy) {
        const int64_t row = ((int64_t)n * a.tiles_y + yy) * a.tiles_x;
        const int lo = a.start[row + max(tx - a.rx, 0)];
        const int hi = a.start[row + tx + 1];
        for (int e0 = lo; e0 < hi; e0 += 64) {
            const int e = e0 + lane;
            bool keep = false;
            float4 rec = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (e < hi) {
                rec = a.sorted[e];
                int c0, c1, r0, r1;
                keep = disc_pixels(rec.x, rec.y, a.r, a.H, a.W, c0, c1, r0, r1) && c1 >= x0 && c0 <= x1 &&
                       r1 >= y0 && r0 <= y1;
            }
            const uint64_t kept = __ballot(keep);
            const int cnt = __popcll(kept);
            if (m + cnt > kPtBatch) {
                pt_batch<KB>(a, L, top, m, live, px, py);
                m = 0;
            }
            if (keep) {
                const int d = m + __popcll(kept & lt_mask);
                L.xy[d] = make_double2((double)rec.x, (double)rec.y);
                L.key[d] = make_key(rec.z, __float_as_int(rec.w));
            }
            m += cnt;
        }
    }
    if (m > 0) pt_batch<KB>(a, L, top, m, live, px, py);
    pt_write<KB, EXACT>(a, L, top, px, py, n, tx, ty);
}

static PtArgs pt_args(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H, int W,
                      float radius, int K, int* hdr, int* start, int* bsum, int* home, int* rank, float4* sorted) {
    PtArgs a;
    a.pts = pts;
    a.first = first;
    a.np = np;
    a.P = P;
    a.N = N;
    a.H = H;
    a.W = W;
    a.K = K;
    a.r = radius;
    a.r2 = (double)radius * (double)radius;
    a.tiles_x = (W + kTile - 1) / kTile;
    a.tiles_y = (H + kTile - 1) / kTile;
    // pixel-range spans of a disc: at most floor(r W + 0.03) columns past its
    // first (the ranges are widened by 0.01 pixel at each end)
    const int span_x = (int)fmin(floor((double)radius * W + 0.05), (double)W);
    const int span_y = (int)fmin(floor((double)radius * H + 0.05), (double)H);
    a.rx = min((kTile - 1 + span_x) / kTile, a.tiles_x - 1);
    a.ry = min((kTile - 1 + span_y) / kTile, a.tiles_y - 1);
    a.T = (int64_t)N * a.tiles_x * a.tiles_y;
    a.hdr = hdr;
    a.start = start;
    a.bsum = bsum;
    a.home = home;
    a.rank = rank;
    a.sorted = sorted;
    a.idx = nullptr;
    a.zbuf = nullptr;
    a.dists = nullptr;
    return a;
}

int64_t pt_scan_blocks(int64_t T) { return (T + kScanTile - 1) / kScanTile; }

static hipError_t pt_sort(const PtArgs& a, hipStream_t s) {
    hipError_t e = launch_fill_i32(a.start, a.T + 1, 0, s);
    if (e != hipSuccess) return e;
    const int64_t nthreads = a.P > a.N ? a.P : a.N;
    const unsigned g = (unsigned)((nthreads + 255) / 256);
    hipLaunchKernelGGL(pt_count_kernel, dim3(g), dim3(256), 0, s, a);
    const int64_t nb = pt_scan_blocks(a.T);
    hipLaunchKernelGGL(pt_scan_sums_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a.start, a.T, a.bsum);
    hipLaunchKernelGGL(pt_scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, a.bsum, nb);
    hipLaunchKernelGGL(pt_scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a.start, a.T, a.bsum, nb);
    if (a.P > 0) hipLaunchKernelGGL(pt_scatter_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int KB, bool EXACT>
static hipError_t pt_fine_k(const PtArgs& a, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    const dim3 grid(a.tiles_x, a.tiles_y, a.N);
    if (eb) (void)hipEventRecord(eb, s);
    hipLaunchKernelGGL((pt_raster_kernel<KB, EXACT>), grid, dim3(64), 0, s, a);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

hipError_t launch_points_fwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, int* hdr, int* start, int* bsum, int* home, int* rank,
                             float4* sorted, int32_t* idx, float* zbuf, float* dists, hipStream_t s, hipEvent_t eb,
                             hipEvent_t ee) {
    PtArgs a = pt_args(pts, P, first, np, N, H, W, radius, K, hdr, start, bsum, home, rank, sorted);
    a.idx = idx;
    a.zbuf = zbuf;
    a.dists = dists;
    hipError_t e = pt_sort(a, s);
    if (e != hipSuccess) return e;
    const bool aligned = (((uintptr_t)idx | (uintptr_t)zbuf | (uintptr_t)dists) & 15) == 0;
#define PT_FINE_BUCKET(KB)                                          \
    if (K <= KB) {                                                  \
        if (K == KB && aligned) return pt_fine_k<KB, true>(a, s, eb, ee); \
        return pt_fine_k<KB, false>(a, s, eb, ee);                  \
    }
    if (K <= 1) return pt_fine_k<1, true>(a, s, eb, ee);
    if (K <= 2) return pt_fine_k<2, true>(a, s, eb, ee);
    PT_FINE_BUCKET(4)
    PT_FINE_BUCKET(8)
    PT_FINE_BUCKET(16)
    PT_FINE_BUCKET(32)
    PT_FINE_BUCKET(64)
#undef PT_FINE_BUCKET
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Backward.  zbuf_k = z_p and dists_k = (x_p - px)^2 + (y_p - py)^2 for the
// point p held in slot k, so dL/dz_p collects grad_zbuf and dL/d(x_p, y_p)
// collects 2 grad_dists (x_p - px, y_p - py) over p's slots.  One thread per
// point, in home-tile order so that the threads of a wave read neighbouring
// pixels: it visits the pixels its disc covers (the forward's exact test),
// finds itself in each pixel's id list and sums its own terms, then writes
// its gradient once.  A point is listed only at pixels its disc covers, so
// no slot is missed, and every gradient is a plain store.
// ---------------------------------------------------------------------------
struct PtBwdArgs {
    const float4* sorted;
    const int* start;
    const int64_t* first;
    const int64_t* np;
    const int32_t* idx;
    const float* gz;
    const float* gd;
    float* grad;
    int* hdr;
    int64_t T;
    int N, H, W, K;
    float r;
    double r2;
    int reuse;
    BinSig sig;
};

__global__ __launch_bounds__(256) void pt_bwd_kernel(PtBwdArgs b) {
    if (b.reuse) {
        bool same = true;
#pragma unroll
        for (int i = 0; i < kSigWords; ++i) same = same && (b.hdr[kHdrSig + i] == b.sig.w[i]);
        if (!same) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&b.hdr[kHdrStatus], kStatReuse);
            return;
        }
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.start[b.T]) return;
    const float4 rec = b.sorted[i];
    const int id = __float_as_int(rec.w);
    const int n = find_mesh(b.first, b.np, b.N, id);
    int c0, c1, r0, r1;
    if (n < 0 || !disc_pixels(rec.x, rec.y, b.r, b.H, b.W, c0, c1, r0, r1)) return;
    const double x = rec.x, y = rec.y;
    double gx = 0.0, gy = 0.0, gzs = 0.0;
    for (int r = r0; r <= r1; ++r) {
        const double py = 1.0 - (double)(2 * r + 1) / (double)b.H;
        for (int c = c0; c <= c1; ++c) {
            const double px = 1.0 - (double)(2 * c + 1) / (double)b.W;
            if (!(pt_d2(x, y, px, py) < b.r2)) continue;
            const int64_t s0 = (((int64_t)n * b.H + r) * b.W + c) * b.K;
            const int32_t* row = b.idx + s0;
            for (int k = 0; k < b.K; ++k) {
                if (row[k] != id) continue;
                if (b.gz) gzs += (double)b.gz[s0 + k];
                if (b.gd) {
                    const double g = 2.0 * (double)b.gd[s0 + k];
                    gx += g * (x - px);
                    gy += g * (y - py);
                }
                break;
            }
        }
    }
    b.grad[3 * (int64_t)id + 0] = (float)gx;
    b.grad[3 * (int64_t)id + 1] = (float)gy;
    b.grad[3 * (int64_t)id + 2] = (float)gzs;
}

hipError_t launch_points_bwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, const int32_t* idx, const float* gz, const float* gd,
                             float* grad, int* hdr, int* start, int* bsum, int* home, int* rank, float4* sorted,
                             bool reuse, const BinSig& sig, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    const PtArgs a = pt_args(pts, P, first, np, N, H, W, radius, K, hdr, start, bsum, home, rank, sorted);
    hipError_t e = launch_fill_f32(grad, 3 * P, 0.0f, s);
    if (e != hipSuccess) return e;
    if (!reuse) {
        e = launch_header_init(hdr, sig, s);
        if (e != hipSuccess) return e;
        e = pt_sort(a, s);
        if (e != hipSuccess) return e;
    }
    if (P == 0) return hipSuccess;
    PtBwdArgs b;
    b.sorted = sorted;
    b.start = start;
    b.first = first;
    b.np = np;
    b.idx = idx;
    b.gz = gz;
    b.gd = gd;
    b.grad = grad;
    b.hdr = hdr;
    b.T = a.T;
    b.N = N;
    b.H = H;
    b.W = W;
    b.K = K;
    b.r = radius;
    b.r2 = a.r2;
    b.reuse = reuse ? 1 : 0;
    b.sig = sig;
    if (eb) (void)hipEventRecord(eb, s);
    hipLaunchKernelGGL(pt_bwd_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, b);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compositing (paper, Section 3.3).  One thread per pixel over its K slots;
// slots whose id is negative (or not below P) take no part.  Opacities come
// either as given or, for splats, from the squared distance: alpha = 1 - d/r^2.
//   Alpha:  out = sum_k alpha_k T_k f_k,  T_k = prod_{j<k} (1 - alpha_j)
//   Norm:   out = sum_k alpha_k f_k / S,   S = sum_k alpha_k (0 where S <= 0)
// Backward (g = upstream gradient of the pixel, g_k = <g, f_k>):
//   Alpha:  dL/dalpha_k = T_k (g_k - R_k),  R_k = sum_{i>k} alpha_i g_i
//           prod_{k<j<i} (1 - alpha_j), which runs backwards as
//           R_{k-1} = alpha_k g_k + (1 - alpha_k) R_k -- no division by
//           1 - alpha_k, so a fully opaque slot is no special case;
//           dL/df_k = alpha_k T_k g.
//   Norm:   dL/dalpha_k = (g_k - <g, out>) / S,  dL/df_k = alpha_k g / S.
// Feature gradients are scattered to the point rows with float atomics.
// ---------------------------------------------------------------------------
struct CompArgs {
    const int32_t* idx;
    const float* w;
    const float* f;
    int64_t P, npix;
    int K, D;
    int norm, from_d;
    float inv_r2;
};

__device__ __forceinline__ float comp_alpha(const CompArgs& a, int64_t o) {
    const float w = a.w[o];
    return a.from_d ? 1.0f - w * a.inv_r2 : w;
}

template <int CB>
__global__ __launch_bounds__(256) void composite_fwd_kernel(CompArgs a, float* __restrict__ img) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npix) return;
    float out[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) out[c] = 0.0f;
    float T = 1.0f, S = 0.0f;
    for (int k = 0; k < a.K; ++k) {
        const int64_t o = p * a.K + k;
        const int id = a.idx[o];
        if (id < 0 || id >= a.P) continue;
        const float al = comp_alpha(a, o);
        const float wk = a.norm ? al : al * T;
        const float* fr = a.f + (int64_t)id * a.D;
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c < a.D) out[c] = fmaf(wk, fr[c], out[c]);
        T *= 1.0f - al;
        S += al;
    }
    const float sc = a.norm ? (S > 0.0f ? 1.0f / S : 0.0f) : 1.0f;
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (c < a.D) img[p * a.D + c] = out[c] * sc;
}

template <int CB>
__global__ __launch_bounds__(256) void composite_bwd_kernel(CompArgs a, const float* __restrict__ gimg,
                                                            float* __restrict__ gw, float* __restrict__ gf) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npix) return;
    float g[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) g[c] = c < a.D ? gimg[p * a.D + c] : 0.0f;
    const float chain = a.from_d ? -a.inv_r2 : 1.0f;
    if (!a.norm) {
        // forward sweep: T_k (kept in gw) and the feature gradients
        float T = 1.0f;
        for (int k = 0; k < a.K; ++k) {
            const int64_t o = p * a.K + k;
            const int id = a.idx[o];
            if (id < 0 || id >= a.P) {
                gw[o] = 0.0f;
                continue;
            }
            const float al = comp_alpha(a, o);
            gw[o] = T;
            if (gf) {
                const float wk = al * T;
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < a.D) atomicAdd(gf + (int64_t)id * a.D + c, wk * g[c]);
            }
            T *= 1.0f - al;
        }
        // backward sweep: R_k and dL/dalpha_k = T_k (g_k - R_k)
        float R = 0.0f;
        for (int k = a.K - 1; k >= 0; --k) {
            const int64_t o = p * a.K + k;
            const int id = a.idx[o];
            if (id < 0 || id >= a.P) continue;
            const float al = comp_alpha(a, o);
            const float* fr = a.f + (int64_t)id * a.D;
            float gk = 0.0f;
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < a.D) gk = fmaf(g[c], fr[c], gk);
            gw[o] = gw[o] * (gk - R) * chain;
            R = fmaf(1.0f - al, R, al * gk);
        }
    } else {
        // first sweep: S, sum alpha_k g_k, and g_k kept in gw
        float S = 0.0f, A = 0.0f;
        for (int k = 0; k < a.K; ++k) {
            const int64_t o = p * a.K + k;
            const int id = a.idx[o];
            if (id < 0 || id >= a.P) {
                gw[o] = 0.0f;
                continue;
            }
            const float al = comp_alpha(a, o);
            const float* fr = a.f + (int64_t)id * a.D;
            float gk = 0.0f;
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < a.D) gk = fmaf(g[c], fr[c], gk);
            gw[o] = gk;
            S += al;
            A = fmaf(al, gk, A);
        }
        const bool lit = S > 0.0f;
        const float invS = lit ? 1.0f / S : 0.0f;
        const float gout = A * invS;
        for (int k = 0; k < a.K; ++k) {
            const int64_t o = p * a.K + k;
            const int id = a.idx[o];
            if (id < 0 || id >= a.P) continue;
            if (!lit) {
                gw[o] = 0.0f;
                continue;
            }
            gw[o] = (gw[o] - gout) * invS * chain;
            if (gf) {
                const float wk = comp_alpha(a, o) * invS;
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < a.D) atomicAdd(gf + (int64_t)id * a.D + c, wk * g[c]);
            }
        }
    }
}

static CompArgs comp_args(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K, int D,
                          int mode, float radius) {
    CompArgs a;
    a.idx = idx;
    a.w = w;
    a.f = f;
    a.P = P;
    a.npix = npix;
    a.K = K;
    a.D = D;
    a.norm = (mode & 1) ? 1 : 0;
    a.from_d = (mode & 2) ? 1 : 0;
    a.inv_r2 = a.from_d ? (float)(1.0 / ((double)radius * (double)radius)) : 0.0f;
    return a;
}

hipError_t launch_composite_fwd(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K,
                                int D, int mode, float radius, float* img, hipStream_t s) {
    if (npix == 0) return hipSuccess;
    const CompArgs a = comp_args(idx, w, f, P, npix, K, D, mode, radius);
    const dim3 grid((unsigned)((npix + 255) / 256));
    if (D <= 4)
        hipLaunchKernelGGL(composite_fwd_kernel<4>, grid, dim3(256), 0, s, a, img);
    else
        hipLaunchKernelGGL(composite_fwd_kernel<8>, grid, dim3(256), 0, s, a, img);
    return hipGetLastError();
}

hipError_t launch_composite_bwd(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K,
                                int D, int mode, float radius, const float* gimg, float* gw, float* gf,
                                hipStream_t s) {
    if (gf) {
        hipError_t e = launch_fill_f32(gf, P * D, 0.0f, s);
        if (e != hipSuccess) return e;
    }
    if (npix == 0) return hipSuccess;
    const CompArgs a = comp_args(idx, w, f, P, npix, K, D, mode, radius);
    const dim3 grid((unsigned)((npix + 255) / 256));
    if (D <= 4)
        hipLaunchKernelGGL(composite_bwd_kernel<4>, grid, dim3(256), 0, s, a, gimg, gw, gf);
    else
        hipLaunchKernelGGL(composite_bwd_kernel<8>, grid, dim3(256), 0, s, a, gimg, gw, gf);
    return hipGetLastError();
}

}  // namespace rast
