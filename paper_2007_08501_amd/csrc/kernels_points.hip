// kernels_points.hip -- point-cloud rasterizer and compositing for gfx950.
//
//   pt_count      cloud id, home tile and rank in that tile of every point
//                 (counts gathered per block in LDS when the tiles fit)
//   pt_scan_*     exclusive scan of the per-tile counts into tile starts
//   pt_scatter    one thread per point: 16-byte record at its sorted slot
//   pt_order_*    tile order for the fine pass, heaviest first
//   pt_raster     one wave per 8x8 tile: candidates from the home lists of
//                 the tiles that can reach it, cull, exact FP64 test over
//                 each candidate's pixel range, K nearest along z in
//                 registers, write the fragments
//   pt_bwd_slots  one workgroup per home tile (device-sized grid): the ids of
//                 the tile's pixel box, matched to the tile's own points
//                 through an LDS hash; each point sums its own slots (no
//                 atomics).  pt_bwd_tile / pt_bwd: the point-major forms
//                 for large radii
//   composite     a pixel's slots over the lanes of a wave segment, four per
//                 lane: Alpha / Norm compositing and its backward
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
    int span_x, span_y;     // pixel columns / rows a disc reaches past its first
    int64_t T;              // tiles in the batch
    int* hdr;
    int* start;             // T+1: counts, then tile starts
    int* bsum;              // scan block sums
    int* home;              // (P) home tile or -1
    int* rank;              // (P) rank within the home tile
    float4* sorted;         // (P) x, y, z, id
    int* order;             // (T) tiles, heaviest first
    int* ohist;             // (64) tile counts per work bucket, then bucket starts, then bucket ends
    int32_t* idx;           // (N,H,W,K) outputs
    float* zbuf;
    float* dists;
};

// Home tile of point p, or -1 when it takes no part (outside every cloud,
// behind the camera, or covering no pixel).
__device__ __forceinline__ int pt_home(const PtArgs& a, int64_t p) {
    const int n = find_mesh(a.first, a.np, a.N, p);
    const float x = a.pts[3 * p], y = a.pts[3 * p + 1], z = a.pts[3 * p + 2];
    int c0, c1, r0, r1;
    if (n < 0 || !(z >= 0.0f) || !disc_pixels(x, y, a.r, a.H, a.W, c0, c1, r0, r1)) return -1;
    return (int)(((int64_t)n * a.tiles_y + r0 / kTile) * a.tiles_x + c0 / kTile);
}

// cloud range check: inside [0, P] and ascending without overlap
__device__ __forceinline__ void pt_check_cloud(const PtArgs& a, int64_t i) {
    const int64_t f = a.first[i], c = a.np[i];
    bool bad = f < 0 || c < 0 || f + c > a.P;
    if (i > 0) bad = bad || f < a.first[i - 1] + a.np[i - 1];
    if (bad) atomicOr(&a.hdr[kHdrStatus], kStatMesh);
}

// Counting, one thread per point: the rank of a point within its home tile is
// the count before its own increment.
__global__ __launch_bounds__(256) void pt_count_kernel(PtArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.N) pt_check_cloud(a, p);
    if (p >= a.P) return;
    const int h = pt_home(a, p);
    a.home[p] = h;
    a.rank[p] = h >= 0 ? atomicAdd(&a.start[h], 1) : 0;
}

// The same with the counts of a block's points first gathered in an LDS
// histogram of every tile of the batch (when they fit): one global atomic per
// tile a block touches instead of one per point.  A point's rank is the
// block's base for its tile plus its rank within the block.
constexpr int kCountThreads = 1024;
constexpr int kCountPer = 8;                  // points per thread
constexpr int kCountLdsTiles = 16384;         // tiles the LDS histogram holds

__global__ __launch_bounds__(kCountThreads) void pt_count_lds_kernel(PtArgs a) {
    __shared__ int hist[kCountLdsTiles];
    const int T = (int)a.T;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < a.N; i += kCountThreads) pt_check_cloud(a, i);
    for (int i = threadIdx.x; i < T; i += kCountThreads) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kCountThreads * kCountPer + threadIdx.x;
    int h[kCountPer], lr[kCountPer];
#pragma unroll
    for (int j = 0; j < kCountPer; ++j) {
        const int64_t p = base + (int64_t)j * kCountThreads;
        h[j] = p < a.P ? pt_home(a, p) : -1;
        lr[j] = h[j] >= 0 ? atomicAdd(&hist[h[j]], 1) : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < T; i += kCountThreads) {
        const int c = hist[i];
        if (c > 0) hist[i] = atomicAdd(&a.start[i], c);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCountPer; ++j) {
        const int64_t p = base + (int64_t)j * kCountThreads;
        if (p < a.P) {
            a.home[p] = h[j];
            a.rank[p] = h[j] >= 0 ? hist[h[j]] + lr[j] : 0;
        }
    }
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

// Tile order for the fine pass, heaviest first: a tile's work is its number
// of candidates (the sorted points of the home tiles that can reach it),
// bucketed on a log scale (two buckets per octave), and a counting sort over
// the 64 buckets lists the tiles.  Within a bucket the order is arbitrary;
// the fragments do not depend on it.
constexpr int kPtOrderBuckets = 64;

__device__ __forceinline__ int pt_tile_bucket(const PtArgs& a, int t) {
    const int per_img = a.tiles_x * a.tiles_y;
    const int n = t / per_img;
    const int tt = t - n * per_img;
    const int ty = tt / a.tiles_x, tx = tt - ty * a.tiles_x;
    int w = 0;
    for (int yy = max(ty - a.ry, 0); yy <= ty; ++yy) {
        const int64_t row = ((int64_t)n * a.tiles_y + yy) * a.tiles_x;
        w += a.start[row + tx + 1] - a.start[row + max(tx - a.rx, 0)];
    }
    const unsigned v = (unsigned)w + 1u;
    const int lg = 31 - __clz(v);
    const int level = min(2 * lg + (lg > 0 ? (int)((v >> (lg - 1)) & 1u) : 0), kPtOrderBuckets - 1);
    return kPtOrderBuckets - 1 - level;  // the last bucket: tiles without candidates
}

__global__ __launch_bounds__(256) void pt_order_hist_kernel(PtArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    (void)wave_bucket_slot(a.ohist, t < a.T ? pt_tile_bucket(a, (int)t) : -1);
}

__global__ void pt_order_scan_kernel(int* __restrict__ ohist) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < kPtOrderBuckets; ++i) {
            const int v = ohist[i];
            ohist[i] = acc;
            acc += v;
        }
    }
}

__global__ __launch_bounds__(256) void pt_order_scatter_kernel(PtArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int pos = wave_bucket_slot(a.ohist, t < a.T ? pt_tile_bucket(a, (int)t) : -1);
    if (t < a.T) a.order[pos] = (int)t;
}

static hipError_t pt_order(const PtArgs& a, hipStream_t s) {
    hipError_t e = launch_fill_i32(a.ohist, kPtOrderBuckets, 0, s);
    if (e != hipSuccess) return e;
    const unsigned g = (unsigned)((a.T + 255) / 256);
    hipLaunchKernelGGL(pt_order_hist_kernel, dim3(g), dim3(256), 0, s, a);
    hipLaunchKernelGGL(pt_order_scan_kernel, dim3(1), dim3(64), 0, s, a.ohist);
    hipLaunchKernelGGL(pt_order_scatter_kernel, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fine pass.  Candidates are gathered a wave-wide chunk at a time, culled on
// their pixel ranges and compacted into an LDS batch; a full batch is tested
// in FP64 over each candidate's pixel range (the squared distance in the
// same operations and order as a plain evaluation, so the decision is
// reproducible bit for bit), the hits are listed per pixel, and each lane's
// list goes through its register top-K eight keys at a time.
// ---------------------------------------------------------------------------
constexpr int kPtLoads = 4;  // candidate chunks loaded at once

// Candidates per batch: larger batches waste less of the last eight-key push
// of each batch, and the 64-key queue's kernel is held to two waves per SIMD
// by its registers anyway; the smaller queues keep a smaller batch, whose
// LDS lets more waves share a compute unit.
template <int KB>
constexpr int pt_batch_size() { return KB >= 64 ? 192 : 128; }

template <int B>
struct PtBatchLds {
    static_assert(B <= 256, "the per-pixel lists hold byte indices");
    static constexpr int kCap = B;
    double2 xy[B];
    uint64_t key[B];                        // (z, id) sort key
    int rng[B];                             // pixel range in the tile: c0 | c1 << 3 | r0 << 6 | r1 << 9
    int cnt[64];                            // hits of each pixel in the batch
    double cx[kTile], cy[kTile];            // FP64 centres of the tile's pixel columns and rows
    unsigned char lst[B * 64];              // entry i of pixel l at [i * 64 + l]
};

// The tile's LDS: the candidate batch, reused at the end to stage one output
// array of the tile (64 pixels x K slots, pixel-major) for the row stores.
template <int KB>
union PtLds {
    PtBatchLds<pt_batch_size<KB>()> b;
    uint32_t stage[64 * KB];
};

__device__ __forceinline__ double pt_d2(double x, double y, double px, double py) {
    const double dx = x - px, dy = y - py;
    return dx * dx + dy * dy;
}

// Pushes a lane's listed hits into its queue, eight at a time, merging
// within the first S slots (S = KB: the whole queue).
template <int S, int KB, class BL>
__device__ __forceinline__ void pt_push_hits(TopK<KB>& top, const BL& L, const unsigned char* my, int nl, int nmax) {
    for (int i0 = 0; i0 < nmax; i0 += 8) {
        uint64_t b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = (i0 + u < nl) ? L.key[my[64 * (i0 + u)]] : kEmptyKey;
        if constexpr (S == KB)
            top.push8(b);
        else
            top.template merge8_prefix<S>(b);
    }
}

// `held`: keys in the lane's queue (at most KB); the queue's keys are its
// first `held` slots, in order.  The coverage tests are made candidate-major:
// a lane takes a candidate and tests only the pixels of its range, listing
// each hit under its pixel; the lists' order depends on the LDS atomics, the
// queues do not (every key is distinct and a queue keeps the smallest ones).
template <int KB, class BL>
__device__ __forceinline__ void pt_batch(const PtArgs& a, BL& L, TopK<KB>& top, int& held, int m) {
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int j = lane; j < m; j += 64) {
        const double2 q = L.xy[j];
        const int g = L.rng[j];
        const int ca = g & 7, cb = (g >> 3) & 7, ra = (g >> 6) & 7, rb = (g >> 9) & 7;
        for (int rr = ra; rr <= rb; ++rr) {
            const double dy = q.y - L.cy[rr];
            for (int cc = ca; cc <= cb; ++cc) {
                const double dx = q.x - L.cx[cc];
                if (dx * dx + dy * dy < a.r2) {
                    const int pix = rr * kTile + cc;
                    const int pos = atomicAdd(&L.cnt[pix], 1);
                    L.lst[pos * 64 + pix] = (unsigned char)j;
                }
            }
        }
    }
    __syncthreads();
    const int nl = L.cnt[lane];
    const unsigned char* my = L.lst + lane;
    const int nmax = wave_max(nl);
    if constexpr (KB >= 16 && is_pow2(KB)) {
        // every push of this batch fits the smallest prefix that holds the
        // wave's largest queue after it (the choice is uniform over the wave)
        const int need = wave_max(held + nl);
        if (need <= 8)
            pt_push_hits<8, KB>(top, L, my, nl, nmax);
        else if (need <= 16)
            pt_push_hits<16, KB>(top, L, my, nl, nmax);
        else if (need <= 32 && KB > 32)
            pt_push_hits<(KB > 32 ? 32 : KB), KB>(top, L, my, nl, nmax);
        else
            pt_push_hits<KB, KB>(top, L, my, nl, nmax);
    } else {
        pt_push_hits<KB, KB>(top, L, my, nl, nmax);
    }
    held = min(held + nl, KB);
    L.cnt[lane] = 0;
    __syncthreads();
}

// Stores one staged output array of the tile: tile row r is the contiguous
// run of cols * K words at out + r * W * K, staged at stage + r * 8 * K, and
// is written by consecutive lanes, 16 bytes each when `vec` (full-width tile,
// W * K a multiple of four, 16-byte aligned outputs).
__device__ __forceinline__ void pt_store_rows(uint32_t* __restrict__ out, const uint32_t* stage, int K, int rowK,
                                              int rows, int cols, bool vec) {
    const int lane = threadIdx.x & 63;
    const int nrow = cols * K;
    for (int r = 0; r < rows; ++r) {
        const uint32_t* src = stage + r * kTile * K;
        uint32_t* dst = out + r * rowK;
        if (vec) {
            for (int e = 4 * lane; e < nrow; e += 256)
                *reinterpret_cast<uint4*>(dst + e) = *reinterpret_cast<const uint4*>(src + e);
        } else {
            for (int e = lane; e < nrow; e += 64) dst[e] = src[e];
        }
    }
}

// Writes the tile's fragments: ids and depths from the keys, squared
// distances recomputed in FP64 exactly as the test evaluated them.
template <int KB, bool EXACT>
__device__ __forceinline__ void pt_write(const PtArgs& a, PtLds<KB>& L, const TopK<KB>& top, double px, double py,
                                         int n, int tx, int ty, bool aligned) {
    const int lane = threadIdx.x & 63;
    const int K = EXACT ? KB : a.K;
    const int rows = min(kTile, a.H - ty * kTile), cols = min(kTile, a.W - tx * kTile);
    const int64_t pix0 = ((int64_t)n * a.H + ty * kTile) * a.W + tx * kTile;
    const int rowK = a.W * K;
    const bool vec = aligned && cols == kTile && (rowK & 3) == 0;
    uint32_t* st = L.stage + lane * K;
    // ids
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (EXACT || k < K) st[k] = top.q[k] == kEmptyKey ? 0xffffffffu : (uint32_t)top.q[k];
    __syncthreads();
    pt_store_rows(reinterpret_cast<uint32_t*>(a.idx + pix0 * K), L.stage, K, rowK, rows, cols, vec);
    __syncthreads();
    // depths
    const uint32_t neg1 = __float_as_uint(-1.0f);
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (EXACT || k < K) st[k] = top.q[k] == kEmptyKey ? neg1 : (uint32_t)(top.q[k] >> 32);
    __syncthreads();
    pt_store_rows(reinterpret_cast<uint32_t*>(a.zbuf + pix0 * K), L.stage, K, rowK, rows, cols, vec);
    __syncthreads();
    // squared distances
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (EXACT || k < K) {
            float d = -1.0f;
            if (top.q[k] != kEmptyKey) {
                const int64_t id = (int64_t)(uint32_t)top.q[k];
                d = (float)pt_d2((double)a.pts[3 * id], (double)a.pts[3 * id + 1], px, py);
            }
            st[k] = __float_as_uint(d);
        }
    }
    __syncthreads();
    pt_store_rows(reinterpret_cast<uint32_t*>(a.dists + pix0 * K), L.stage, K, rowK, rows, cols, vec);
}

// At least two waves per SIMD: left alone, the compiler takes more than half
// the register file for the 64-key queue (one wave per SIMD), and the pass
// runs a quarter slower than with the few spills the bound costs.
template <int KB, bool EXACT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void pt_raster_kernel(PtArgs a, bool aligned) {
    __shared__ PtLds<KB> L;
    // workgroups start in launch order, so the tiles are taken heaviest first
    const int t = a.order[blockIdx.x];
    const int per_img = a.tiles_x * a.tiles_y;
    const int n = t / per_img;
    const int tt = t - n * per_img;
    const int ty = tt / a.tiles_x, tx = tt - ty * a.tiles_x;
    const int lane = threadIdx.x & 63;
    const int r = ty * kTile + (lane >> 3), c = tx * kTile + (lane & 7);
    const double px = 1.0 - (double)(2 * c + 1) / (double)a.W;
    const double py = 1.0 - (double)(2 * r + 1) / (double)a.H;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int x1 = min(x0 + kTile, a.W) - 1, y1 = min(y0 + kTile, a.H) - 1;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // pixel centres as in a plain evaluation (the first batch's barrier
    // publishes them); columns or rows past the image edge are never tested
    if (lane < kTile)
        L.b.cx[lane] = 1.0 - (double)(2 * (x0 + lane) + 1) / (double)a.W;
    else if (lane < 2 * kTile)
        L.b.cy[lane - kTile] = 1.0 - (double)(2 * (y0 + lane - kTile) + 1) / (double)a.H;
    L.b.cnt[lane] = 0;

    TopK<KB> top;
    top.init();
    int held = 0;
    int m = 0;
    for (int yy = max(ty - a.ry, 0); yy <= ty; ++yy) {
        const int64_t row = ((int64_t)n * a.tiles_y + yy) * a.tiles_x;
        const int lo = a.start[row + max(tx - a.rx, 0)];
        const int hi = a.start[row + tx + 1];
        // kPtLoads chunks of candidates are loaded before any is culled, so
        // their loads overlap
        for (int e0 = lo; e0 < hi; e0 += 64 * kPtLoads) {
            float4 recs[kPtLoads];
#pragma unroll
            for (int u = 0; u < kPtLoads; ++u) {
                const int e = e0 + 64 * u + lane;
                recs[u] = e < hi ? a.sorted[e] : make_float4(0.0f, 0.0f, -1.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kPtLoads; ++u) {
                if (e0 + 64 * u >= hi) break;  // uniform
                const float4 rec = recs[u];
                bool keep = false;
                int c0 = 0, c1 = 0, r0 = 0, r1 = 0;
                if (e0 + 64 * u + lane < hi) {
                    keep = disc_pixels(rec.x, rec.y, a.r, a.H, a.W, c0, c1, r0, r1) && c1 >= x0 && c0 <= x1 &&
                           r1 >= y0 && r0 <= y1;
                }
                const uint64_t kept = __ballot(keep);
                const int cnt = __popcll(kept);
                if (m + cnt > L.b.kCap) {
                    pt_batch<KB>(a, L.b, top, held, m);
                    m = 0;
                }
                if (keep) {
                    const int d = m + __popcll(kept & lt_mask);
                    L.b.xy[d] = make_double2((double)rec.x, (double)rec.y);
                    L.b.key[d] = make_key(rec.z, __float_as_int(rec.w));
                    L.b.rng[d] = (max(c0, x0) - x0) | ((min(c1, x1) - x0) << 3) | ((max(r0, y0) - y0) << 6) |
                                 ((min(r1, y1) - y0) << 9);
                }
                m += cnt;
            }
        }
    }
    if (m > 0) pt_batch<KB>(a, L.b, top, held, m);
    __syncthreads();
    pt_write<KB, EXACT>(a, L, top, px, py, n, tx, ty, aligned);
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
    a.span_x = (int)fmin(floor((double)radius * W + 0.05), (double)W);
    a.span_y = (int)fmin(floor((double)radius * H + 0.05), (double)H);
    a.rx = min((kTile - 1 + a.span_x) / kTile, a.tiles_x - 1);
    a.ry = min((kTile - 1 + a.span_y) / kTile, a.tiles_y - 1);
    a.T = (int64_t)N * a.tiles_x * a.tiles_y;
    a.hdr = hdr;
    a.start = start;
    a.bsum = bsum;
    a.home = home;
    a.rank = rank;
    a.sorted = sorted;
    a.order = nullptr;
    a.ohist = nullptr;
    a.idx = nullptr;
    a.zbuf = nullptr;
    a.dists = nullptr;
    return a;
}

int64_t pt_scan_blocks(int64_t T) { return (T + kScanTile - 1) / kScanTile; }

static hipError_t pt_sort(const PtArgs& a, hipStream_t s) {
    hipError_t e = launch_fill_i32(a.start, a.T + 1, 0, s);
    if (e != hipSuccess) return e;
    if (a.T <= kCountLdsTiles) {
        const int64_t per_block = (int64_t)kCountThreads * kCountPer;
        const unsigned g = (unsigned)((a.P + per_block - 1) / per_block);
        hipLaunchKernelGGL(pt_count_lds_kernel, dim3(g > 0 ? g : 1), dim3(kCountThreads), 0, s, a);
    } else {
        const int64_t nthreads = a.P > a.N ? a.P : a.N;
        const unsigned g = (unsigned)((nthreads + 255) / 256);
        hipLaunchKernelGGL(pt_count_kernel, dim3(g), dim3(256), 0, s, a);
    }
    const int64_t nb = pt_scan_blocks(a.T);
    hipLaunchKernelGGL(pt_scan_sums_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a.start, a.T, a.bsum);
    hipLaunchKernelGGL(pt_scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, a.bsum, nb);
    hipLaunchKernelGGL(pt_scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a.start, a.T, a.bsum, nb);
    if (a.P > 0) hipLaunchKernelGGL(pt_scatter_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int KB, bool EXACT>
static hipError_t pt_fine_k(const PtArgs& a, bool aligned, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    const dim3 grid((unsigned)a.T);
    if (eb) (void)hipEventRecord(eb, s);
    hipLaunchKernelGGL((pt_raster_kernel<KB, EXACT>), grid, dim3(64), 0, s, a, aligned);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

hipError_t launch_points_fwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, int* hdr, int* start, int* bsum, int* home, int* rank,
                             float4* sorted, int* order, int* ohist, int32_t* idx, float* zbuf, float* dists,
                             hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    PtArgs a = pt_args(pts, P, first, np, N, H, W, radius, K, hdr, start, bsum, home, rank, sorted);
    a.order = order;
    a.ohist = ohist;
    a.idx = idx;
    a.zbuf = zbuf;
    a.dists = dists;
    hipError_t e = pt_sort(a, s);
    if (e != hipSuccess) return e;
    e = pt_order(a, s);
    if (e != hipSuccess) return e;
    const bool aligned = (((uintptr_t)idx | (uintptr_t)zbuf | (uintptr_t)dists) & 15) == 0;
#define PT_FINE_BUCKET(KB)                                                     \
    if (K <= KB) {                                                             \
        if (K == KB) return pt_fine_k<KB, true>(a, aligned, s, eb, ee);        \
        return pt_fine_k<KB, false>(a, aligned, s, eb, ee);                    \
    }
    if (K <= 1) return pt_fine_k<1, true>(a, aligned, s, eb, ee);
    if (K <= 2) return pt_fine_k<2, true>(a, aligned, s, eb, ee);
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
// collects 2 grad_dists (x_p - px, y_p - py) over p's slots.  Every point
// gathers its own terms and writes its gradient once (no atomics, the same
// sum order on every run): it visits the pixels its disc covers (the
// forward's exact test) and finds itself in each pixel's id list.  A point is
// listed only at pixels its disc covers, so no slot is missed.
//
// One workgroup per home tile: the points of the tile are contiguous in the
// sorted array, and every pixel they can cover lies in the tile grown by the
// disc reach (span_x columns to the right, span_y rows down), so the ids and
// upstream gradients of that pixel box are staged in LDS first (rows padded
// to a multiple of four slots for 16-byte reads).  When the box does not fit
// in LDS, a one-thread-per-point form reads the lists from global memory.
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
    const int* order;  // tiles, most candidates first (the forward's order)
    const int* ohist;  // bucket ends of that order
    int64_t T;
    int N, H, W, K;
    float r;
    double r2;
    int tiles_x, tiles_y, span_x, span_y;
    int Kp;  // slots per pixel in LDS (K rounded up to a multiple of 4)
    int reuse;
    BinSig sig;
};

__device__ __forceinline__ bool pt_bwd_usable(const PtBwdArgs& b) {
    if (!b.reuse) return true;
    bool same = true;
#pragma unroll
    for (int i = 0; i < kSigWords; ++i) same = same && (b.hdr[kHdrSig + i] == b.sig.w[i]);
    if (!same && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&b.hdr[kHdrStatus], kStatReuse);
    return same;
}

__device__ __forceinline__ void pt_write_grad(const PtBwdArgs& b, int id, double gx, double gy, double gzs) {
    b.grad[3 * (int64_t)id + 0] = (float)gx;
    b.grad[3 * (int64_t)id + 1] = (float)gy;
    b.grad[3 * (int64_t)id + 2] = (float)gzs;
}

// One thread per sorted point, id lists read from global memory.
__global__ __launch_bounds__(256) void pt_bwd_kernel(PtBwdArgs b) {
    if (!pt_bwd_usable(b)) return;
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
    pt_write_grad(b, id, gx, gy, gzs);
}

constexpr int kBwdTileThreads = 256;
constexpr int64_t kLdsPerCu = 160 * 1024;

// e / d for 0 <= e < 2^22 and d > 0: the float estimate is off by at most one.
__device__ __forceinline__ int small_div(int e, int d, float inv_d) {
    int q = (int)((float)e * inv_d);
    if (q * d > e) --q;
    else if ((q + 1) * d <= e) ++q;
    return q;
}
extern __shared__ uint32_t bwd_lds[];

__device__ __forceinline__ void pt_bwd_tile(const PtBwdArgs& b, int t) {
    const int lo = b.start[t], hi = b.start[t + 1];
    if (lo == hi) return;  // uniform: no point has this home tile
    const int per_img = b.tiles_x * b.tiles_y;
    const int n = t / per_img;
    const int rem = t - n * per_img;
    const int ty = rem / b.tiles_x, tx = rem - (rem / b.tiles_x) * b.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int bw = min(x0 + kTile + b.span_x, b.W) - x0;
    const int bh = min(y0 + kTile + b.span_y, b.H) - y0;
    const int K = b.K, Kp = b.Kp;
    const int box = bw * bh * Kp;
    int* sidx = reinterpret_cast<int*>(bwd_lds);
    float* sgz = reinterpret_cast<float*>(bwd_lds + box);
    float* sgd = reinterpret_cast<float*>(bwd_lds + (b.gz ? 2 : 1) * box);
    // stage the box: LDS word e = (row * bw + pixel) * Kp + slot; padding
    // slots hold -1.  Eight words per thread are loaded before any is stored.
    const int rowl = bw * Kp, nbox = bh * rowl;
    const float inv_rowl = 1.0f / (float)rowl, inv_kp = 1.0f / (float)Kp;
    for (int e0 = 0; e0 < nbox; e0 += 8 * kBwdTileThreads) {
        int vi[8];
        float vz[8], vd[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = e0 + j * kBwdTileThreads + (int)threadIdx.x;
            vi[j] = -1;
            vz[j] = vd[j] = 0.0f;
            if (e < nbox) {
                const int r = small_div(e, rowl, inv_rowl);
                const int rem = e - r * rowl;
                const int px = small_div(rem, Kp, inv_kp);
                const int k = rem - px * Kp;
                if (k < K) {
                    const int64_t g = (((int64_t)n * b.H + y0 + r) * b.W + x0 + px) * K + k;
                    vi[j] = b.idx[g];
                    if (b.gz) vz[j] = b.gz[g];
                    if (b.gd) vd[j] = b.gd[g];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = e0 + j * kBwdTileThreads + (int)threadIdx.x;
            if (e < nbox) {
                sidx[e] = vi[j];
                if (b.gz) sgz[e] = vz[j];
                if (b.gd) sgd[e] = vd[j];
            }
        }
    }
    __syncthreads();
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBwdTileThreads) {
        const float4 rec = b.sorted[i];
        const int id = __float_as_int(rec.w);
        int c0, c1, r0, r1;
        disc_pixels(rec.x, rec.y, b.r, b.H, b.W, c0, c1, r0, r1);
        // the ranges lie in the box by construction of the home tile and the
        // reach; clamping only keeps every LDS index in bounds
        r0 = max(r0, y0);
        c0 = max(c0, x0);
        r1 = min(r1, y0 + bh - 1);
        c1 = min(c1, x0 + bw - 1);
        const double x = rec.x, y = rec.y;
        double gx = 0.0, gy = 0.0, gzs = 0.0;
        for (int r = r0; r <= r1; ++r) {
            const double py = 1.0 - (double)(2 * r + 1) / (double)b.H;
            for (int c = c0; c <= c1; ++c) {
                const double px = 1.0 - (double)(2 * c + 1) / (double)b.W;
                if (!(pt_d2(x, y, px, py) < b.r2)) continue;
                const int l0 = ((r - y0) * bw + (c - x0)) * Kp;
                int s = -1;
                for (int k4 = 0; k4 < K && s < 0; k4 += 4) {
                    const int4 v = *reinterpret_cast<const int4*>(sidx + l0 + k4);
                    s = v.x == id ? l0 + k4 : v.y == id ? l0 + k4 + 1 : v.z == id ? l0 + k4 + 2
                        : v.w == id ? l0 + k4 + 3 : -1;
                }
                if (s < 0) continue;
                if (b.gz) gzs += (double)sgz[s];
                if (b.gd) {
                    const double g = 2.0 * (double)sgd[s];
                    gx += g * (x - px);
                    gy += g * (y - py);
                }
            }
        }
        pt_write_grad(b, id, gx, gy, gzs);
    }
}

// A device-sized grid walks the tiles that have candidates (a point's home
// tile is among its own candidates), most loaded first; tiles with no home
// point are skipped.
__global__ __launch_bounds__(kBwdTileThreads) void pt_bwd_tile_kernel(PtBwdArgs b) {
    if (!pt_bwd_usable(b)) return;
    const int ntile = b.ohist[kPtOrderBuckets - 2];
    for (int j = blockIdx.x; j < ntile; j += gridDim.x) {
        pt_bwd_tile(b, b.order[j]);
        __syncthreads();  // the next tile restages the LDS box
    }
}

// Slot-major form of the same backward.  Every slot that names a point lies
// in that point's pixel range, hence in the box of its home tile, so each
// slot is claimed by exactly one tile.  A tile hashes its own points (id ->
// local index) in LDS, reads its box of slots in coalesced rows, and notes
// for each slot naming one of its points the slot's k in a per-point cell of
// the pixel's offset within the point's pixel range; a point is listed at
// most once per pixel, so every cell has one writer and no atomics are
// needed.  Each point then sums its cells in row-major pixel order in FP64,
// as the point-major form does.  Points beyond kSlotCap per tile are taken in
// chunks, each rescanning the box.
constexpr int kSlotCap = 1024;          // points per chunk
constexpr int kSlotHash = 2 * kSlotCap; // hash entries (power of two)
constexpr int kSlotMaxCells = 25;       // (span_x + 1) * (span_y + 1) at most
constexpr int kSlotLoads = 16;          // slots loaded per thread before any is used
constexpr uint8_t kNoSlot = 0xff;

static_assert(kSlotHash == 1 << 11, "slot_hash yields 11 bits");
__device__ __forceinline__ int slot_hash(int id) { return (int)(((uint32_t)id * 2654435761u) >> 21); }

__device__ __forceinline__ void pt_bwd_slots_tile(const PtBwdArgs& b, int t, int2* htab, int* prc, uint8_t* cell) {
    const int lo = b.start[t], hi = b.start[t + 1];
    if (lo == hi) return;  // uniform: no point has this home tile
    const int per_img = b.tiles_x * b.tiles_y;
    const int n = t / per_img;
    const int rem = t - n * per_img;
    const int ty = rem / b.tiles_x, tx = rem - ty * b.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int bw = min(x0 + kTile + b.span_x, b.W) - x0;
    const int bh = min(y0 + kTile + b.span_y, b.H) - y0;
    const int K = b.K;
    const int ex = b.span_x + 1, ey = b.span_y + 1, ncell = ex * ey;
    const int rowl = bw * K, nbox = bh * rowl;
    const float inv_rowl = 1.0f / (float)rowl, inv_k = 1.0f / (float)K;
    for (int c_lo = lo; c_lo < hi; c_lo += kSlotCap) {
        const int nloc = min(kSlotCap, hi - c_lo);
        for (int i = threadIdx.x; i < kSlotHash; i += kBwdTileThreads) htab[i] = make_int2(-1, 0);
        uint32_t* cw = reinterpret_cast<uint32_t*>(cell);
        for (int i = threadIdx.x; i < (nloc * ncell + 3) / 4; i += kBwdTileThreads) cw[i] = 0xffffffffu;
        __syncthreads();
        for (int i = threadIdx.x; i < nloc; i += kBwdTileThreads) {
            const float4 rec = b.sorted[c_lo + i];
            const int id = __float_as_int(rec.w);
            int c0, c1, r0, r1;
            disc_pixels(rec.x, rec.y, b.r, b.H, b.W, c0, c1, r0, r1);
            prc[i] = max(r0, y0) | (max(c0, x0) << 16);
            // ids are distinct, and the table is at least half empty
            for (int h = slot_hash(id);; h = (h + 1) & (kSlotHash - 1)) {
                if (atomicCAS(&htab[h].x, -1, id) == -1) {
                    htab[h].y = i;
                    break;
                }
            }
        }
        __syncthreads();
        for (int e0 = 0; e0 < nbox; e0 += kSlotLoads * kBwdTileThreads) {
            int vi[kSlotLoads];
#pragma unroll
            for (int j = 0; j < kSlotLoads; ++j) {
                const int e = e0 + j * kBwdTileThreads + (int)threadIdx.x;
                vi[j] = -1;
                if (e < nbox) {
                    const int r = small_div(e, rowl, inv_rowl);
                    const int q = e - r * rowl;
                    const int64_t g = ((int64_t)n * b.H + y0 + r) * b.W * K + (int64_t)x0 * K + q;
                    vi[j] = b.idx[g];
                }
            }
#pragma unroll
            for (int j = 0; j < kSlotLoads; ++j) {
                const int id = vi[j];
                if (id < 0) continue;
                int local = -1;
                for (int h = slot_hash(id);; h = (h + 1) & (kSlotHash - 1)) {
                    const int2 en = htab[h];
                    if (en.x == id) {
                        local = en.y;
                        break;
                    }
                    if (en.x < 0) break;
                }
                if (local < 0) continue;  // another tile's point, or another chunk's
                const int e = e0 + j * kBwdTileThreads + (int)threadIdx.x;
                const int r = small_div(e, rowl, inv_rowl);
                const int q = e - r * rowl;
                const int c = small_div(q, K, inv_k);
                const int k = q - c * K;
                const int pr = prc[local];
                const int dr = y0 + r - (pr & 0xffff), dc = x0 + c - (pr >> 16);
                if (dr < 0 || dr >= ey || dc < 0 || dc >= ex) continue;  // outside the point's pixel range
                cell[local * ncell + dr * ex + dc] = (uint8_t)k;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nloc; i += kBwdTileThreads) {
            const float4 rec = b.sorted[c_lo + i];
            const int id = __float_as_int(rec.w);
            const int pr = prc[i];
            const int pr0 = pr & 0xffff, pc0 = pr >> 16;
            const double x = rec.x, y = rec.y;
            double gx = 0.0, gy = 0.0, gzs = 0.0;
            const uint8_t* mine = cell + i * ncell;
            for (int dr = 0; dr < ey; ++dr) {
                const int r = pr0 + dr;
                const double py = 1.0 - (double)(2 * r + 1) / (double)b.H;
                for (int dc = 0; dc < ex; ++dc) {
                    const int k = mine[dr * ex + dc];
                    if (k == kNoSlot) continue;
                    const int c = pc0 + dc;
                    const double px = 1.0 - (double)(2 * c + 1) / (double)b.W;
                    const int64_t g = (((int64_t)n * b.H + r) * b.W + c) * K + k;
                    if (b.gz) gzs += (double)b.gz[g];
                    if (b.gd) {
                        const double gg = 2.0 * (double)b.gd[g];
                        gx += gg * (x - px);
                        gy += gg * (y - py);
                    }
                }
            }
            pt_write_grad(b, id, gx, gy, gzs);
        }
        __syncthreads();  // the next chunk or tile clears the tables
    }
}

__global__ __launch_bounds__(kBwdTileThreads) void pt_bwd_slots_kernel(PtBwdArgs b) {
    if (!pt_bwd_usable(b)) return;
    int2* htab = reinterpret_cast<int2*>(bwd_lds);
    int* prc = reinterpret_cast<int*>(htab + kSlotHash);
    uint8_t* cell = reinterpret_cast<uint8_t*>(prc + kSlotCap);
    const int ntile = b.ohist[kPtOrderBuckets - 2];
    for (int j = blockIdx.x; j < ntile; j += gridDim.x) pt_bwd_slots_tile(b, b.order[j], htab, prc, cell);
}

// LDS bytes of the slot-major backward, or 0 when its cells do not fit.
static size_t pt_bwd_slots_lds_bytes(int span_x, int span_y, int K) {
    const int64_t ncell = (int64_t)(span_x + 1) * (span_y + 1);
    if (ncell > kSlotMaxCells || K >= kNoSlot) return 0;
    return (size_t)kSlotHash * sizeof(int2) + (size_t)kSlotCap * sizeof(int) +
           (((size_t)kSlotCap * ncell + 3) & ~(size_t)3);
}

// LDS bytes of the box-staged backward, or 0 when it does not fit.
static size_t pt_bwd_lds_bytes(const PtArgs& a, int span_x, int span_y, bool gz, bool gd) {
    const int64_t bw = min(kTile + span_x, a.W), bh = min(kTile + span_y, a.H);
    const int64_t Kp = (a.K + 3) & ~3;
    const int64_t bytes = bw * bh * Kp * 4 * (1 + (gz ? 1 : 0) + (gd ? 1 : 0));
    return bytes <= 65536 ? (size_t)bytes : 0;
}

hipError_t launch_points_bwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, const int32_t* idx, const float* gz, const float* gd,
                             float* grad, int* hdr, int* start, int* bsum, int* home, int* rank, float4* sorted,
                             int* order, int* ohist, int n_cus, bool reuse, const BinSig& sig, hipStream_t s,
                             hipEvent_t eb, hipEvent_t ee) {
    PtArgs a = pt_args(pts, P, first, np, N, H, W, radius, K, hdr, start, bsum, home, rank, sorted);
    a.order = order;
    a.ohist = ohist;
    hipError_t e = launch_fill_f32(grad, 3 * P, 0.0f, s);
    if (e != hipSuccess) return e;
    if (!reuse) {
        e = launch_header_init(hdr, sig, s);
        if (e != hipSuccess) return e;
        e = pt_sort(a, s);
        if (e != hipSuccess) return e;
        e = pt_order(a, s);
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
    b.order = order;
    b.ohist = ohist;
    b.T = a.T;
    b.N = N;
    b.H = H;
    b.W = W;
    b.K = K;
    b.r = radius;
    b.r2 = a.r2;
    b.tiles_x = a.tiles_x;
    b.tiles_y = a.tiles_y;
    b.span_x = a.span_x;
    b.span_y = a.span_y;
    b.Kp = (K + 3) & ~3;
    b.reuse = reuse ? 1 : 0;
    b.sig = sig;
    const size_t slds = pt_bwd_slots_lds_bytes(a.span_x, a.span_y, K);
    const size_t lds = pt_bwd_lds_bytes(a, a.span_x, a.span_y, gz != nullptr, gd != nullptr);
    if (eb) (void)hipEventRecord(eb, s);
    if (slds > 0) {
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, kLdsPerCu / (int64_t)slds));
        const int64_t grid = std::min<int64_t>(a.T, (int64_t)std::max(n_cus, 1) * per_cu);
        hipLaunchKernelGGL(pt_bwd_slots_kernel, dim3((unsigned)grid), dim3(kBwdTileThreads), slds, s, b);
    } else if (lds > 0) {
        // as many workgroups as the compute units hold at once (LDS-bound)
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, kLdsPerCu / (int64_t)lds));
        const int64_t grid = std::min<int64_t>(a.T, (int64_t)std::max(n_cus, 1) * per_cu);
        hipLaunchKernelGGL(pt_bwd_tile_kernel, dim3((unsigned)grid), dim3(kBwdTileThreads), lds, s, b);
    }
    else
        hipLaunchKernelGGL(pt_bwd_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, b);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compositing (paper, Section 3.3).  A pixel's K slots are spread over L
// lanes of a wave, four consecutive slots per lane (L the power of two with
// 4 L >= K, 64 / L pixels per wave): each lane combines its own four slots in
// order and only the per-lane aggregates cross lanes, in segmented scans of
// log2(L) steps.  Slots whose id is negative (or not below P) take no part.
// Opacities come either as given or, for splats, from the squared distance:
// alpha = 1 - d/r^2.
//   Alpha:  out = sum_k alpha_k T_k f_k,  T_k = prod_{j<k} (1 - alpha_j)
//   Norm:   out = sum_k alpha_k f_k / S,   S = sum_k alpha_k (0 where S <= 0)
// Backward (g = upstream gradient of the pixel, g_k = <g, f_k>):
//   Alpha:  dL/dalpha_k = T_k (g_k - R_k),  R_k = sum_{i>k} alpha_i g_i
//           prod_{k<j<i} (1 - alpha_j).  R_k is the composition of the affine
//           maps x -> (1 - alpha_i) x + alpha_i g_i over the slots after k,
//           applied to 0 -- a suffix scan with no division by 1 - alpha_k, so
//           a fully opaque slot is no special case;  dL/df_k = alpha_k T_k g.
//   Norm:   dL/dalpha_k = (g_k - <g, out>) / S,  dL/df_k = alpha_k g / S.
// Feature gradients are scattered to the point rows with float atomics.  With
// no feature table every feature is 1 (silhouette compositing) and nothing is
// gathered.
// ---------------------------------------------------------------------------
constexpr int kCompQ = 4;  // consecutive slots per lane
// four words at 4-byte alignment (one 16-byte global load)
typedef int i32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef float f32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

struct CompArgs {
    const int32_t* idx;
    const float* w;
    const float* f;  // (P, D) features, or nullptr: all ones
    int64_t P, npix;
    int K, D;
    int norm, from_d;
    float inv_r2;
};

// The lane's slots of pixel p: point ids (-1 if a slot takes no part) and opacities (0 then).
__device__ __forceinline__ void comp_slots(const CompArgs& a, int64_t p, int sub, int (&id)[kCompQ],
                                           float (&al)[kCompQ]) {
    int32_t iv[kCompQ];
    float wv[kCompQ];
    const int64_t o = p * a.K + kCompQ * sub;
    if (p < a.npix && kCompQ * (sub + 1) <= a.K) {
        // the lane's four slots as one 16-byte load per array (4-byte
        // aligned: a pixel's slots start at any word)
        const i32x4_a4 vi = *reinterpret_cast<const i32x4_a4*>(a.idx + o);
        const f32x4_a4 vw = *reinterpret_cast<const f32x4_a4*>(a.w + o);
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            iv[i] = vi[i];
            wv[i] = vw[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            const bool in = p < a.npix && kCompQ * sub + i < a.K;
            iv[i] = in ? a.idx[o + i] : -1;
            wv[i] = in ? a.w[o + i] : 0.0f;
        }
    }
#pragma unroll
    for (int i = 0; i < kCompQ; ++i) {
        const bool ok = iv[i] >= 0 && iv[i] < a.P;
        id[i] = ok ? iv[i] : -1;
        al[i] = ok ? (a.from_d ? 1.0f - wv[i] * a.inv_r2 : wv[i]) : 0.0f;
    }
}

// exclusive product over the lower lanes of the segment
template <int L>
__device__ __forceinline__ float seg_exclusive_prod(float t, int sub) {
#pragma unroll
    for (int d = 1; d < L; d <<= 1) {
        const float u = __shfl_up(t, d, L);
        if (sub >= d) t *= u;
    }
    const float e = __shfl_up(t, 1, L);
    return sub == 0 ? 1.0f : e;
}

template <int L>
__device__ __forceinline__ float seg_sum(float v) {
#pragma unroll
    for (int d = L / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, L);
    return v;
}

template <int L, int CB>
__global__ __launch_bounds__(256) void composite_fwd_kernel(CompArgs a, float* __restrict__ img) {
    constexpr int PPW = 64 / L;
    const int lane = threadIdx.x & 63, sub = lane & (L - 1), grp = lane / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p0 = wave * PPW; p0 < a.npix; p0 += nwaves * PPW) {
        const int64_t p = p0 + grp;
        int id[kCompQ];
        float al[kCompQ];
        comp_slots(a, p, sub, id, al);
        float t = 1.0f, S = 0.0f;
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            t *= 1.0f - al[i];
            S += al[i];
        }
        float T = a.norm ? 1.0f : seg_exclusive_prod<L>(t, sub);
        float acc[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            if (id[i] >= 0) {
                const float wk = a.norm ? al[i] : al[i] * T;
                if (a.f) {
                    const float* fr = a.f + (int64_t)id[i] * a.D;
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c < a.D) acc[c] = fmaf(wk, fr[c], acc[c]);
                } else {
#pragma unroll
                    for (int c = 0; c < CB; ++c) acc[c] += wk;  // features all ones
                }
            }
            T *= 1.0f - al[i];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c < a.D) acc[c] = seg_sum<L>(acc[c]);
        if (a.norm) S = seg_sum<L>(S);
        const float sc = a.norm ? (S > 0.0f ? 1.0f / S : 0.0f) : 1.0f;
        if (sub == 0 && p < a.npix) {
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < a.D) img[p * a.D + c] = acc[c] * sc;
        }
    }
}

template <int L, int CB>
__global__ __launch_bounds__(256) void composite_bwd_kernel(CompArgs a, const float* __restrict__ gimg,
                                                            float* __restrict__ gw, float* __restrict__ gf) {
    constexpr int PPW = 64 / L;
    const int lane = threadIdx.x & 63, sub = lane & (L - 1), grp = lane / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const float chain = a.from_d ? -a.inv_r2 : 1.0f;
    for (int64_t p0 = wave * PPW; p0 < a.npix; p0 += nwaves * PPW) {
        const int64_t p = p0 + grp;
        int id[kCompQ];
        float al[kCompQ];
        comp_slots(a, p, sub, id, al);
        float g[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) g[c] = (p < a.npix && c < a.D) ? gimg[p * a.D + c] : 0.0f;
        float gk[kCompQ];
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            gk[i] = 0.0f;
            if (id[i] >= 0) {
                if (a.f) {
                    const float* fr = a.f + (int64_t)id[i] * a.D;
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c < a.D) gk[i] = fmaf(g[c], fr[c], gk[i]);
                } else {
#pragma unroll
                    for (int c = 0; c < CB; ++c) gk[i] += g[c];  // features all ones
                }
            }
        }
        float dal[kCompQ], wf[kCompQ];
        if (!a.norm) {
            float t = 1.0f;
#pragma unroll
            for (int i = 0; i < kCompQ; ++i) t *= 1.0f - al[i];
            float T = seg_exclusive_prod<L>(t, sub);
            // the lane's four maps composed (slot 4 sub outermost), then the
            // composition of every later lane's maps: a suffix scan
            float A = 1.0f, B = 0.0f;
#pragma unroll
            for (int i = kCompQ - 1; i >= 0; --i) {
                B = fmaf(1.0f - al[i], B, al[i] * gk[i]);
                A *= 1.0f - al[i];
            }
#pragma unroll
            for (int d = 1; d < L; d <<= 1) {
                const float A2 = __shfl_down(A, d, L), B2 = __shfl_down(B, d, L);
                if (sub + d < L) {
                    B = fmaf(A, B2, B);
                    A *= A2;
                }
            }
            const float Bn = __shfl_down(B, 1, L);
            float V = sub == L - 1 ? 0.0f : Bn;  // R after the lane's last slot
            float R[kCompQ];
#pragma unroll
            for (int i = kCompQ - 1; i >= 0; --i) {
                R[i] = V;
                V = fmaf(1.0f - al[i], V, al[i] * gk[i]);
            }
#pragma unroll
            for (int i = 0; i < kCompQ; ++i) {
                dal[i] = T * (gk[i] - R[i]);
                wf[i] = al[i] * T;
                T *= 1.0f - al[i];
            }
        } else {
            float S = 0.0f, Ag = 0.0f;
#pragma unroll
            for (int i = 0; i < kCompQ; ++i) {
                S += al[i];
                Ag = fmaf(al[i], gk[i], Ag);
            }
            S = seg_sum<L>(S);
            Ag = seg_sum<L>(Ag);
            const float invS = S > 0.0f ? 1.0f / S : 0.0f;
#pragma unroll
            for (int i = 0; i < kCompQ; ++i) {
                dal[i] = (gk[i] - Ag * invS) * invS;
                wf[i] = al[i] * invS;
            }
        }
        const int64_t o = p * a.K + kCompQ * sub;
        if (p < a.npix && kCompQ * (sub + 1) <= a.K) {
            f32x4_a4 v;
#pragma unroll
            for (int i = 0; i < kCompQ; ++i) v[i] = id[i] >= 0 ? dal[i] * chain : 0.0f;
            *reinterpret_cast<f32x4_a4*>(gw + o) = v;  // one 16-byte store
        } else {
#pragma unroll
            for (int i = 0; i < kCompQ; ++i)
                if (p < a.npix && kCompQ * sub + i < a.K) gw[o + i] = id[i] >= 0 ? dal[i] * chain : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < kCompQ; ++i) {
            if (gf && id[i] >= 0 && wf[i] != 0.0f) {
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < a.D) atomicAdd(gf + (int64_t)id[i] * a.D + c, wf[i] * g[c]);
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

// Workgroups of a grid-stride launch: one wave per 64 / L pixels, at most
// 2048 workgroups of four waves.
static unsigned comp_blocks(int64_t npix, int L) {
    const int64_t waves = (npix + 64 / L - 1) / (64 / L);
    const int64_t blocks = (waves + 3) / 4;
    return (unsigned)(blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks));
}

template <int CB>
static hipError_t comp_launch(const CompArgs& a, bool bwd, const float* gimg, float* gw, float* gf, float* img,
                              hipStream_t s) {
#define COMP_L(L)                                                                                      \
    if (a.K <= kCompQ * L) {                                                                           \
        const dim3 grid(comp_blocks(a.npix, L));                                                       \
        if (bwd)                                                                                       \
            hipLaunchKernelGGL((composite_bwd_kernel<L, CB>), grid, dim3(256), 0, s, a, gimg, gw, gf); \
        else                                                                                           \
            hipLaunchKernelGGL((composite_fwd_kernel<L, CB>), grid, dim3(256), 0, s, a, img);          \
        return hipGetLastError();                                                                      \
    }
    COMP_L(1)
    COMP_L(2)
    COMP_L(4)
    COMP_L(8)
    COMP_L(16)
#undef COMP_L
    return hipErrorInvalidValue;
}

hipError_t launch_composite_fwd(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K,
                                int D, int mode, float radius, float* img, hipStream_t s) {
    if (npix == 0) return hipSuccess;
    const CompArgs a = comp_args(idx, w, f, P, npix, K, D, mode, radius);
    if (D <= 4) return comp_launch<4>(a, false, nullptr, nullptr, nullptr, img, s);
    return comp_launch<8>(a, false, nullptr, nullptr, nullptr, img, s);
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
    if (D <= 4) return comp_launch<4>(a, true, gimg, gw, gf, nullptr, s);
    return comp_launch<8>(a, true, gimg, gw, gf, nullptr, s);
}

}  // namespace rast
