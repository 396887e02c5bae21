// kernels_fwd.hip -- forward rasterization kernels for gfx950.
//
//   face_setup      one thread per face: mesh id, 112-byte record, padded bbox
//   bin_faces       one thread per face: append the face to every bin its bbox
//                   touches (counting only when lists == nullptr); largest bin
//                   count -> workspace header, overflow flag
//   raster_tiles    one wave per 8x8 pixel tile: loop over candidate faces
//                   (all faces of the tile's mesh, or the tile's bin list),
//                   cull per tile, test per pixel, keep the K nearest in
//                   registers, write the fragments
//
// The paper's rasterizer (Section 3.2) first works on image tiles to drop
// faces and then on pixels, keeping per-pixel queues of the K nearest faces;
// this is that scheme laid out for 64-wide waves.
#include "../../include/rast.h"
#include "device.hpp"
#include "launch.hpp"
#include "tile_layout.hpp"

namespace rast {

__global__ void fill_i32_kernel(int* __restrict__ p, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void fill_f32_kernel(float* __restrict__ p, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Clears the workspace header and stamps the binning signature.
__global__ void header_init_kernel(int* __restrict__ hdr, BinSig sig) {
    for (int i = threadIdx.x; i < kHdrWords; i += blockDim.x)
        hdr[i] = (i >= kHdrSig && i < kHdrSig + kSigWords) ? sig.w[i - kHdrSig] : 0;
}

hipError_t launch_header_init(int* hdr, const BinSig& sig, hipStream_t s) {
    hipLaunchKernelGGL(header_init_kernel, dim3(1), dim3(64), 0, s, hdr, sig);
    return hipGetLastError();
}

// The header's status bits as a rast_status code (the same precedence as
// rast_query_status) and its largest bin count, for a caller without a workspace.
__global__ void status_out_kernel(const int* __restrict__ hdr, int32_t* __restrict__ out) {
    if (threadIdx.x == 0) {
        const int h = hdr[kHdrStatus];
        out[0] = (h & kStatMesh) ? RAST_EMESH : ((h & kStatOverflow) ? RAST_EOVERFLOW : RAST_OK);
        out[1] = hdr[kHdrMaxCount];
    }
}

hipError_t launch_status_out(const int* hdr, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(status_out_kernel, dim3(1), dim3(64), 0, s, hdr, out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// One thread per face builds the face's record (make_rec: mesh id, exact FP64
// edge vectors, grown box); the workgroup's 256 records are staged in LDS and
// stored with coalesced 16-byte writes (a lane storing its own 112 bytes
// leaves each store instruction scattered over 64 lines).  The threads below
// N also check the mesh ranges.
__global__ __launch_bounds__(256) void face_setup_kernel(const float* __restrict__ verts, int64_t V,
                                                         const int32_t* __restrict__ faces, int64_t F,
                                                         const int64_t* __restrict__ first,
                                                         const int64_t* __restrict__ nf, int N, float rb, int opts,
                                                         FaceRec* __restrict__ recs, int* __restrict__ hdr) {
    __shared__ FaceRec srec[256];
    const int64_t f0 = (int64_t)blockIdx.x * blockDim.x;
    int64_t f = f0 + threadIdx.x;
    if (first != nullptr && f < N) {
        // mesh range check: inside [0, F] and ascending without overlap
        int64_t a = first[f], c = nf[f];
        bool bad = a < 0 || c < 0 || a + c > F;
        if (f > 0) bad = bad || a < first[f - 1] + nf[f - 1];
        if (bad) atomicOr(&hdr[kHdrStatus], kStatMesh);
    }
    if (f0 >= F) return;  // (uniform over the workgroup)
    if (f < F) {
        int mesh = first != nullptr ? find_mesh(first, nf, N, f) : 0;
        int i0 = faces[3 * f + 0], i1 = faces[3 * f + 1], i2 = faces[3 * f + 2];
        bool idx_ok = i0 >= 0 && i0 < V && i1 >= 0 && i1 < V && i2 >= 0 && i2 < V;
        if (!idx_ok) {
            atomicOr(&hdr[kHdrStatus], kStatMesh);
            mesh = -1;
            i0 = i1 = i2 = 0;
        }
        if (V == 0) {
            srec[threadIdx.x] = make_rec(0, 0, 0, 0, 0, 0, 0, 0, 0, rb, -1);
        } else {
            const float* a = verts + 3 * (int64_t)i0;
            const float* b = verts + 3 * (int64_t)i1;
            const float* c = verts + 3 * (int64_t)i2;
            srec[threadIdx.x] = make_rec(a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2], rb, mesh, opts);
        }
    }
    __syncthreads();
    // the workgroup's records are contiguous: coalesced 16-byte stores
    const int n = (int)min((int64_t)blockDim.x, F - f0);
    const float4* src = reinterpret_cast<const float4*>(srec);
    float4* dst = reinterpret_cast<float4*>(recs + f0);
    constexpr int W4 = sizeof(FaceRec) / sizeof(float4);
    for (int i = threadIdx.x; i < n * W4; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_face_setup(const float* verts, int64_t V, const int32_t* faces, int64_t F, const int64_t* first,
                             const int64_t* nf, int N, float rb, int opts, FaceRec* recs, int* hdr, hipStream_t s) {
    int64_t n = F > N ? F : N;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(face_setup_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, verts, V, faces, F,
                       first, nf, N, rb, opts, recs, hdr);
    return hipGetLastError();
}

// One thread per face appends the face to every bin of its range.  The
// workgroup's 256 consecutive faces (usually neighbours on the mesh, sharing
// bins) first count their appends per distinct bin in an LDS hash table; one
// global atomic per distinct bin then reserves room for all of the
// workgroup's appends to it, and a second walk over the ranges hands out the
// positions.  An append whose bin finds the table full reserves its own
// position with a global atomic, and so does one whose bin is not within
// kBinProbe slots of its hash position (both walks probe the same slots, so
// they agree on which bins the table holds): a workgroup of large faces,
// touching thousands of bins, then costs at most kBinProbe probes per
// append.  The workgroup also records the largest
// count it leaves in any of its bins (the last reservation in a bin ends at
// its final count, so the maximum over workgroups is the largest bin count)
// and flags a count above the capacity M.
constexpr int kBinHash = 1024;  // LDS hash entries of the binning workgroup
constexpr int kBinProbe = 32;   // slots probed per append
__device__ __forceinline__ uint32_t bin_hash(int64_t b) {
    return ((uint32_t)b * 2654435761u ^ (uint32_t)(b >> 32)) >> (32 - 10);
}
static_assert(kBinHash == 1024, "bin_hash yields 10 bits");

__global__ __launch_bounds__(256) void bin_faces_kernel(const FaceRec* __restrict__ recs, int64_t F, int H, int W,
                                                        int bs, int nby, int nbx, int M, int* __restrict__ counts,
                                                        int* __restrict__ lists, int* __restrict__ hdr) {
    __shared__ unsigned long long hkey[kBinHash];  // bin + 1 (0: empty)
    __shared__ int wmax[4];
    __shared__ int hcnt[kBinHash];   // appends per bin, then the next rank to hand out
    __shared__ int hbase[kBinHash];  // the workgroup's reserved start in the bin
    for (int i = threadIdx.x; i < kBinHash; i += blockDim.x) {
        hkey[i] = 0ull;
        hcnt[i] = 0;
    }
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0, bx0 = 0, by0 = 0, nbw = 1, nb = 0;
    if (f < F) {
        const FaceRec& R = recs[f];
        int bx1, by1;
        if (R.ok() && face_bins_of_box(R.bb, H, W, bs, bx0, bx1, by0, by1)) {
            n = R.mesh();
            nbw = bx1 - bx0 + 1;
            nb = nbw * (by1 - by0 + 1);
        }
    }
    __syncthreads();
    // 1. count per distinct bin
    {
        int ri = 0, rj = 0;
        for (int i = 0; i < nb; ++i) {
            const long long bin = ((int64_t)n * nby + by0 + ri) * nbx + bx0 + rj;
            if (++rj == nbw) {
                rj = 0;
                ++ri;
            }
            const unsigned long long key = (unsigned long long)bin + 1ull;
            uint32_t h = bin_hash(bin);
            for (int probe = 0; probe < kBinProbe; ++probe) {
                const unsigned long long prev = atomicCAS(&hkey[h], 0ull, key);
                if (prev == 0ull || prev == key) {
                    atomicAdd(&hcnt[h], 1);
                    break;
                }
                h = (h + 1) & (kBinHash - 1);
            }
        }
    }
    __syncthreads();
    // 2. one reservation per distinct bin
    int top = 0;  // largest count this thread leaves in a bin
    for (int i = threadIdx.x; i < kBinHash; i += blockDim.x) {
        const unsigned long long key = hkey[i];
        if (key != 0ull) {
            hbase[i] = atomicAdd(&counts[key - 1], hcnt[i]);
            top = max(top, hbase[i] + hcnt[i]);
            hcnt[i] = 0;
        }
    }
    __syncthreads();
    // 3. positions
    {
        int ri = 0, rj = 0;
        for (int i = 0; i < nb; ++i) {
            const long long bin = ((int64_t)n * nby + by0 + ri) * nbx + bx0 + rj;
            if (++rj == nbw) {
                rj = 0;
                ++ri;
            }
            const unsigned long long want = (unsigned long long)bin + 1ull;
            uint32_t h = bin_hash(bin);
            int pos = -1;
            for (int probe = 0; probe < kBinProbe; ++probe) {
                const unsigned long long key = hkey[h];
                if (key == want) {
                    pos = hbase[h] + atomicAdd(&hcnt[h], 1);
                    break;
                }
                if (key == 0ull) break;
                h = (h + 1) & (kBinHash - 1);
            }
            if (pos < 0) {
                pos = atomicAdd(&counts[bin], 1);  // (not in the table)
                top = max(top, pos + 1);
            }
            if (lists != nullptr && pos < M) lists[bin * M + pos] = (int)f;
        }
    }
    // the workgroup's largest count: one word per wave, then one read and, only
    // if larger, one atomic per workgroup (same-address atomics serialise)
    for (int o = 32; o > 0; o >>= 1) top = max(top, __shfl_xor(top, o));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = top;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) top = max(top, wmax[w]);
        if (top > __hip_atomic_load(&hdr[kHdrMaxCount], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&hdr[kHdrMaxCount], top);
        if (M > 0 && top > M) atomicOr(&hdr[kHdrStatus], kStatOverflow);
    }
}

hipError_t launch_binning(const FaceRec* recs, int64_t F, int N, int H, int W, int bs, int M, int* counts, int* lists,
                          int* hdr, hipStream_t s) {
    int nby = (H + bs - 1) / bs, nbx = (W + bs - 1) / bs;
    int64_t nbins = (int64_t)N * nby * nbx;
    hipError_t e = launch_fill_i32(counts, nbins, 0, s);
    if (e != hipSuccess) return e;
    if (F > 0) {
        hipLaunchKernelGGL(bin_faces_kernel, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, s, recs, F, H, W, bs, nby,
                           nbx, M, counts, lists, hdr);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fine pass.  One 64-thread workgroup = one wave = one 8x8 tile of image n.
// Faces come either from the whole mesh (BINNED = false) or from the list of
// the bin that contains the tile.  Every face is first culled against the
// tile's extent (a wave-uniform branch) and then tested by each lane for its
// own pixel; winners go through the register top-K.
// ---------------------------------------------------------------------------
struct FineArgs {
    const FaceRec* recs;
    const int64_t* first;
    const int64_t* nf;
    const int* counts;
    const int* lists;
    int64_t F;
    int N, H, W, K;
    float blur;
    int opts;  // rasterizer options (kOpt*)
    int bs, nby, nbx, M;
    int tiles_x, tiles_y;
    int32_t* p2f;
    float* zbuf;
    float* bary;
    float* dists;
};

// LDS of one tile's wave: a chunk of up to 64 candidate faces that overlap the
// tile (the gather gives every lane one list entry, so a chunk is exactly one
// wave wide), and the room the write-out staging needs beyond them.
constexpr int kChunk = tile_layout::kChunk;

// A face as the tile pass keeps it in LDS: the geometry the pixel tests read
// (the fields of FaceRec that the evaluation uses), the face id, and the
// tile's pixels that the face's grown box may cover, as a 64-bit mask
// (bit r*8 + c), which replaces the box.
struct TileRec {
    double2 pa, ab, ac;
    double E;
    float az, dz1, dz2, invE, il0, il1, il2;
    int fid;
    uint64_t mask;
};
static_assert(sizeof(TileRec) == tile_layout::kTileRecBytes, "tile record layout");

struct TileLds {
    TileRec rec[kChunk];
    unsigned char spare[tile_layout::kSpareBytes];  // (staging of the write-out)
};
static_assert(sizeof(TileLds) == tile_layout::kLdsBytes, "tile LDS layout");

// Writes the tile's fragments from the per-lane queues.  Values are staged in
// LDS per pixel and then stored by consecutive lanes to consecutive
// addresses, so every store instruction writes whole contiguous runs (one
// tile row of pix_to_face is 8*K contiguous words) instead of 64 scattered
// words; written slot by slot, each cache line would be completed by K
// separate instructions with loads in between and could be evicted half
// written.  Ids and depths come straight from the keys; barycentrics and
// distances are recomputed from the face records.
constexpr int kStageG1 = tile_layout::kStageG1;  // slots per pass for ids and depths
constexpr int kStageG2 = tile_layout::kStageG2;  // slots per pass for barycentrics and distances

// EXACT: K equals the bucket size KB, so every group width, stride and index
// below is a compile-time constant (the common case); otherwise K < KB is a
// run-time value.  Addresses are 32-bit offsets from the tile's first
// fragment, a wave-uniform base.
// OPT: the rasterizer options that change barycentrics and depth are on
// (a separate instantiation, so that the default path carries no test for them).
// Non-temporal 16-byte stores (the "nt" hint: streamed past the caches).
// The id and depth passes write whole lines (a tile row of either array is
// 8 K contiguous words), so streaming them leaves L2 to the face records the
// tile waves share; the barycentric and distance passes write part lines
// per pass and are stored normally, so that L2 completes their lines.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef int nt_i4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void nt_store(int4 v, int* p) {
    const nt_i4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_i4*>(p));
}
__device__ __forceinline__ void nt_store(float4 v, float* p) {
    const nt_f4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f4*>(p));
}

template <int KB, bool EXACT, bool OPT>
__device__ __forceinline__ void write_fragments(const FineArgs& a, TileLds& L, const TopK<KB>& top, const Pix& p,
                                                int n, int tx, int ty) {
    const int lane = threadIdx.x & 63;
    const int K = EXACT ? KB : a.K;
    const int rows = min(kTile, a.H - ty * kTile), cols = min(kTile, a.W - tx * kTile);
    const int64_t pix0 = ((int64_t)n * a.H + ty * kTile) * a.W + tx * kTile;
    const int rowK = a.W * K;  // fragments per image row
    // EXACT with K a multiple of 4 (the launcher also checked that the four
    // outputs are 16-byte aligned): 16-byte stores of four slots
    constexpr bool V4 = EXACT && (KB % 4 == 0);
    int32_t* const p2f_t = a.p2f + pix0 * K;
    float* const zbuf_t = a.zbuf + pix0 * K;
    float* const dist_t = a.dists + pix0 * K;
    float* const bary_t = a.bary + pix0 * K * 3;
    static_assert(sizeof(TileLds) >= sizeof(float) * 64 * 2 * (kStageG1 + 1), "id/depth staging exceeds the tile LDS");
    static_assert(sizeof(TileLds) >= sizeof(float) * 64 * (4 * kStageG2 + 2), "bary/dist staging exceeds the tile LDS");
    float* stage = reinterpret_cast<float*>(&L);
    // ids and depths
    {
        constexpr int G = KB < kStageG1 ? KB : kStageG1;
        constexpr int S = G + 1;  // odd stride: lane-major writes hit distinct banks
        int* sid = reinterpret_cast<int*>(stage);
        float* sz = stage + 64 * S;
#pragma unroll
        for (int g0 = 0; g0 < KB; g0 += G) {
            if (g0 >= K) continue;  // K is uniform: the whole wave skips
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint64_t key = top.q[g0 + k];
                const bool empty = key == kEmptyKey;
                sid[lane * S + k] = empty ? -1 : (int)(uint32_t)key;
                sz[lane * S + k] = empty ? -1.0f : __uint_as_float((uint32_t)(key >> 32));
            }
            __syncthreads();
            if constexpr (V4) {
                // four consecutive slots of one pixel per lane and store
                constexpr int Q = G / 4;
#pragma unroll
                for (int e0 = 0; e0 < 64 * Q; e0 += 64) {
                    const int e = e0 + lane;
                    const int px = e / Q, q = e - px * Q;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) {
                        const int o = r * rowK + c * K + g0 + 4 * q;
                        const int* si = sid + px * S + 4 * q;
                        const float* zi = sz + px * S + 4 * q;
                        nt_store(make_int4(si[0], si[1], si[2], si[3]), p2f_t + o);
                        nt_store(make_float4(zi[0], zi[1], zi[2], zi[3]), zbuf_t + o);
                    }
                }
            } else {
                const int gw = min(G, K - g0);
                const float inv = 1.0f / (float)gw;
#pragma unroll
                for (int e0 = 0; e0 < 64 * G; e0 += 64) {
                    const int e = e0 + lane;
                    if (e >= 64 * gw) break;
                    const int px = EXACT ? e / gw : stage_pixel(e, inv);
                    const int k = e - px * gw;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) {
                        const int o = r * rowK + c * K + g0 + k;
                        p2f_t[o] = sid[px * S + k];
                        zbuf_t[o] = sz[px * S + k];
                    }
                }
            }
            __syncthreads();
        }
    }
    // barycentrics and signed distances
    {
        constexpr int G = KB < kStageG2 ? KB : kStageG2;
        constexpr int SB = 3 * G + 1, SD = G + 1;
        float* sb = stage;
        float* sd = stage + 64 * SB;
#pragma unroll
        for (int g0 = 0; g0 < KB; g0 += G) {
            if (g0 >= K) continue;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint64_t key = top.q[g0 + k];
                float w0 = -1.0f, w1 = -1.0f, w2 = -1.0f, d = -1.0f;
                if (key != kEmptyKey) {
                    const FaceRec R = a.recs[(uint32_t)key];
                    Eval ev;
                    eval_full(R, p, ev);
                    w0 = ev.w0;
                    w1 = ev.w1;
                    w2 = ev.w2;
                    if (OPT) {
                        float zf;
                        apply_opts(a.opts, R.az, R.dz1, R.dz2, w0, w1, w2, zf);
                    }
                    d = ev.inside ? -ev.d2 : ev.d2;
                }
                sb[lane * SB + 3 * k + 0] = w0;
                sb[lane * SB + 3 * k + 1] = w1;
                sb[lane * SB + 3 * k + 2] = w2;
                sd[lane * SD + k] = d;
            }
            __syncthreads();
            if constexpr (V4) {
                constexpr int QB = 3 * G / 4, QD = G / 4;
#pragma unroll
                for (int e0 = 0; e0 < 64 * QB; e0 += 64) {
                    const int e = e0 + lane;
                    const int px = e / QB, q = e - px * QB;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) {
                        const float* bi = sb + px * SB + 4 * q;
                        *reinterpret_cast<float4*>(bary_t + 3 * (r * rowK + c * K + g0) + 4 * q) =
                            make_float4(bi[0], bi[1], bi[2], bi[3]);
                    }
                }
#pragma unroll
                for (int e0 = 0; e0 < 64 * QD; e0 += 64) {
                    const int e = e0 + lane;
                    const int px = e / QD, q = e - px * QD;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) {
                        const float* di = sd + px * SD + 4 * q;
                        *reinterpret_cast<float4*>(dist_t + r * rowK + c * K + g0 + 4 * q) =
                            make_float4(di[0], di[1], di[2], di[3]);
                    }
                }
            } else {
                const int gw = min(G, K - g0);
                const float inv3 = 1.0f / (float)(3 * gw), inv1 = 1.0f / (float)gw;
#pragma unroll
                for (int e0 = 0; e0 < 64 * 3 * G; e0 += 64) {
                    const int e = e0 + lane;
                    if (e >= 64 * 3 * gw) break;
                    const int px = EXACT ? e / (3 * gw) : stage_pixel(e, inv3);
                    const int m = e - px * 3 * gw;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) bary_t[3 * (r * rowK + c * K + g0) + m] = sb[px * SB + m];
                }
#pragma unroll
                for (int e0 = 0; e0 < 64 * G; e0 += 64) {
                    const int e = e0 + lane;
                    if (e >= 64 * gw) break;
                    const int px = EXACT ? e / gw : stage_pixel(e, inv1);
                    const int k = e - px * gw;
                    const int r = px >> 3, c = px & 7;
                    if (r < rows && c < cols) dist_t[r * rowK + c * K + g0 + k] = sd[px * SD + k];
                }
            }
            __syncthreads();
        }
    }
}

// Transpose of the 64x64 bit matrix whose row i is lane i's word: bit i of
// lane p's result is bit p of lane i's word.  Six butterfly stages: at stage
// j the lanes i and i ^ j exchange the off-diagonal j x j blocks of their
// 2j x 2j block (the lane with bit j clear keeps its low groups of j bits
// and takes the partner's low groups into its high ones, the other keeps its
// high groups and takes the partner's high groups into its low ones).
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
    constexpr uint64_t kLow[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0f0f0f0f0f0f0f0full,
                                  0x00ff00ff00ff00ffull, 0x0000ffff0000ffffull, 0x00000000ffffffffull};
#pragma unroll
    for (int s = 5; s >= 0; --s) {
        const int j = 1 << s;
        const uint64_t m = kLow[s];
        const uint64_t y = __shfl_xor(x, j);
        x = (lane & j) ? ((x & ~m) | ((y & ~m) >> j)) : ((x & m) | ((y & m) << j));
    }
    return x;
}

// One wave rasterizes one 8x8 tile in three steps per chunk of 64 faces:
//  1. gather the chunk's face records, keep those whose box (narrowed by the
//     edge lines) may cover a pixel of the tile (wave ballot + prefix count
//     compacts them into LDS), each with its 64-bit mask of such pixels;
//  2. transpose the kept faces' masks across the wave (lane j holds record
//     j's mask), so that lane p holds the chunk's faces that may cover pixel p;
//  3. every lane walks only its own faces, runs the full test and inserts
//     the faces that count into its register top-K.
// Step 3 is where the arithmetic is; gathering each pixel's candidates first
// keeps lanes from idling on faces that miss their pixel.
template <int KB, bool BINNED, bool EXACT, bool OPT>
__device__ __forceinline__ void raster_tile(const FineArgs& a, TileLds& L, int n, int tx, int ty) {
    const int lane = threadIdx.x & 63;
    const int r = ty * kTile + (lane >> 3);
    const int c = tx * kTile + (lane & 7);
    const Pix p = make_pix(r, c, a.H, a.W);
    // extent of the tile's pixel centres (x decreases with c, y with r), less a
    // margin so that the float test never rejects what the pixel ranges keep
    const int c_last = min(tx * kTile + kTile - 1, a.W - 1);
    const int r_last = min(ty * kTile + kTile - 1, a.H - 1);
    const float mx = 0.1f / (float)a.W, my = 0.1f / (float)a.H;  // 0.05 px, looser than pix_range (0.01 px)
    const float tx_hi = pix_x(tx * kTile, a.W) + mx, tx_lo = pix_x(c_last, a.W) - mx;
    const float ty_hi = pix_y(ty * kTile, a.H) + my, ty_lo = pix_y(r_last, a.H) - my;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // radius beyond which a pixel outside an edge line cannot count (see edge_mask)
    const double rg = (double)sqrtf(a.blur) * (1.0 + 1e-4) + 1e-6;

    TopK<KB> top;
    top.init();

    const int* list = nullptr;
    int64_t base = 0, cnt = 0;
    if (BINNED) {
        int bx = (tx * kTile) / a.bs, by = (ty * kTile) / a.bs;
        int64_t bin = ((int64_t)n * a.nby + by) * a.nbx + bx;
        cnt = min(a.counts[bin], a.M);
        list = a.lists + bin * a.M;
    } else {
        int64_t lo = a.first[n], hi = a.first[n] + a.nf[n];
        lo = lo < 0 ? 0 : lo;
        hi = hi > a.F ? a.F : hi;
        base = lo;
        cnt = hi > lo ? hi - lo : 0;
    }
    for (int64_t c0 = 0; c0 < cnt; c0 += kChunk) {
        // 1. gather and compact the chunk's faces that overlap the tile
        const int64_t e = c0 + lane;
        const bool in_list = e < cnt;
        const int fid = in_list ? (BINNED ? list[e] : (int)(base + e)) : 0;
        // the record as seven 16-byte words (pa | ab | ac | E, a.z, mesh |
        // dz1, dz2, 1/E, il0 | il1, il2, pad | grown box)
        static_assert(sizeof(FaceRec) == 7 * sizeof(float4), "face record layout");
        const float4* rsrc = reinterpret_cast<const float4*>(a.recs + (in_list ? fid : (BINNED ? list[0] : (int)base)));
        const float4 rv0 = rsrc[0], rv1 = rsrc[1], rv2 = rsrc[2], rv3 = rsrc[3], rv4 = rsrc[4], rv5 = rsrc[5];
        const float4 rv6 = rsrc[6];
        uint64_t pm = in_list ? tile_mask(rv6, a.H, a.W, tx * kTile, ty * kTile, tx_lo, tx_hi, ty_lo, ty_hi) : 0ull;
        if (pm != 0ull) {
            // narrow the box's pixels to those near or inside the triangle
            const EdgeGeo G{f4_as_d2(rv0), f4_as_d2(rv1), f4_as_d2(rv2), f4_as_d2(rv3).x};
            pm &= edge_mask(G, rg, a.H, a.W, tx * kTile, ty * kTile);
        }
        const bool keep = pm != 0ull;
        const uint64_t kept = __ballot(keep);
        const int m = __popcll(kept);
        if (keep) {
            const int dst = __popcll(kept & lt_mask);
            float4* rdst = reinterpret_cast<float4*>(&L.rec[dst]);
            rdst[0] = rv0;
            rdst[1] = rv1;
            rdst[2] = rv2;
            rdst[3] = make_float4(rv3.x, rv3.y, rv3.z, rv4.x);  // E | a.z, dz1
            rdst[4] = make_float4(rv4.y, rv4.z, rv4.w, rv5.x);  // dz2, 1/E, il0, il1
            rdst[5] = make_float4(rv5.y, __int_as_float(fid), __uint_as_float((uint32_t)pm),
                                  __uint_as_float((uint32_t)(pm >> 32)));  // il2, id, mask
        }
        __syncthreads();
        // 2. per lane, the faces whose boxes may contain the lane's pixel: lane
        //    j holds kept face j's pixel mask (row j of a 64x64 bit matrix);
        //    the transpose gives lane p the faces of pixel p
        uint64_t mine = lane < m ? L.rec[lane].mask : 0ull;
        mine = transpose64(mine, lane);
        const int nl = __popcll(mine);
        // 3. full test of the lane's own candidates, eight per round; the
        //    round count is the wave's longest list, so the loop is uniform
        //    and the queue stays in place across rounds
        const int nmax = wave_max(nl);
        for (int i0 = 0; i0 < nmax; i0 += 8) {
            uint64_t b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                uint64_t key = kEmptyKey;
                if (mine != 0ull) {
                    const int j = __ffsll((unsigned long long)mine) - 1;
                    mine &= mine - 1;
                    float z;
                    if (face_counts_in_box(L.rec[j], p, a.blur, z, OPT ? a.opts : 0)) key = make_key(z, L.rec[j].fid);
                }
                b[u] = key;
            }
            top.push8(b);
        }
        __syncthreads();
    }
    write_fragments<KB, EXACT, OPT>(a, L, top, p, n, tx, ty);
}

// EXACT: faces_per_pixel equals the queue size KB (chosen at launch).
// The grid's workgroups are taken as tiles in image-major raster order, each
// XCD a contiguous range of them (xcd_item).
template <int KB, bool BINNED, bool EXACT, bool OPT>
__global__ __launch_bounds__(64) void raster_tiles_kernel(FineArgs a) {
    __shared__ TileLds L;
    const int64_t per_img = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t wg = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    const int64_t t = xcd_item(wg, per_img * a.N);
    const int n = (int)(t / per_img);
    const int rem = (int)(t - n * per_img);
    const int ty = rem / a.tiles_x;
    raster_tile<KB, BINNED, EXACT, OPT>(a, L, n, rem - ty * a.tiles_x, ty);
}

// Persistent form: a device-sized grid; each wave pulls the next tile id from
// a counter in the workspace header.  order[] lists tile ids (image-major
// linear ids) most-loaded bins first.  Every wave leaves when the counter
// passes the number of tiles.
// One tile of the persistent form, kept out of line: inlined into the work
// loop, the tile's loop-invariant address arithmetic is hoisted out of it and
// held live across tiles, far beyond the register file.
template <int KB, bool EXACT, bool OPT>
__device__ __noinline__ void raster_tile_persistent(const FineArgs& a, TileLds& L, int n, int tx, int ty) {
    raster_tile<KB, true, EXACT, OPT>(a, L, n, tx, ty);
}

template <int KB, bool EXACT, bool OPT>
__global__ __launch_bounds__(64) void raster_persistent_kernel(FineArgs a, const int* __restrict__ order,
                                                               int* __restrict__ hdr, int total) {
    __shared__ TileLds L;
    for (;;) {
        int item = 0;
        if ((threadIdx.x & 63) == 0) item = atomicAdd(&hdr[kHdrWorkNext], 1);
        item = __shfl(item, 0);
        if (item >= total) break;
        int t = order[item];
        int per_img = a.tiles_x * a.tiles_y;
        int n = t / per_img;
        int rem = t - n * per_img;
        int ty = rem / a.tiles_x;
        int tx = rem - ty * a.tiles_x;
        raster_tile_persistent<KB, EXACT, OPT>(a, L, n, tx, ty);
    }
}

// order[]: tiles sorted by the count of their bin, descending, using a
// counting sort over count buckets (64 buckets of width ceil((M+1)/64)), with
// one global atomic per distinct bucket of a wave (per-thread atomics on the
// 64 counters serialised: about 1 ms at config 3).
__device__ __forceinline__ int tile_bucket(const int* __restrict__ counts, int t, int tiles_x, int tiles_y, int bs,
                                           int nby, int nbx, int M) {
    const int per_img = tiles_x * tiles_y;
    const int n = t / per_img;
    const int rem = t - n * per_img;
    const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
    const int64_t bin = ((int64_t)n * nby + (ty * kTile) / bs) * nbx + (tx * kTile) / bs;
    const int cnt = min(counts[bin], M);
    const int width = (M + 64) / 64;
    return 63 - min(cnt / width, 63);  // bucket 0 = heaviest
}

__global__ __launch_bounds__(256) void order_hist_kernel(const int* __restrict__ counts, int N, int tiles_x,
                                                         int tiles_y, int bs, int nby, int nbx, int M,
                                                         int* __restrict__ hist) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)N * tiles_x * tiles_y;
    (void)wave_bucket_slot(hist, t < total ? tile_bucket(counts, (int)t, tiles_x, tiles_y, bs, nby, nbx, M) : -1);
}

__global__ __launch_bounds__(256) void order_scatter_kernel(const int* __restrict__ counts, int N, int tiles_x,
                                                            int tiles_y, int bs, int nby, int nbx, int M,
                                                            int* __restrict__ hist_off, int* __restrict__ order) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)N * tiles_x * tiles_y;
    const int pos =
        wave_bucket_slot(hist_off, t < total ? tile_bucket(counts, (int)t, tiles_x, tiles_y, bs, nby, nbx, M) : -1);
    if (t < total) order[pos] = (int)t;
}

// exclusive scan of the 64 bucket sizes, in place; also arms the work counter
__global__ void order_scan_kernel(int* __restrict__ hist, int* __restrict__ hdr, int total) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < 64; ++i) {
            int v = hist[i];
            hist[i] = acc;
            acc += v;
        }
        hdr[kHdrWorkNext] = 0;
        hdr[kHdrWorkTotal] = total;
    }
}

template <int KB, bool EXACT, bool OPT>
static hipError_t launch_fine_k(const FineArgs& a, bool binned, int sched, int* order, int* hist, int* hdr,
                                int n_workers, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    if (binned && sched == 1) {
        int total = a.N * a.tiles_x * a.tiles_y;
        hipError_t e = launch_fill_i32(hist, 64, 0, s);
        if (e != hipSuccess) return e;
        unsigned g = (unsigned)((total + 255) / 256);
        hipLaunchKernelGGL(order_hist_kernel, dim3(g), dim3(256), 0, s, a.counts, a.N, a.tiles_x, a.tiles_y, a.bs,
                           a.nby, a.nbx, a.M, hist);
        hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, s, hist, hdr, total);
        hipLaunchKernelGGL(order_scatter_kernel, dim3(g), dim3(256), 0, s, a.counts, a.N, a.tiles_x, a.tiles_y, a.bs,
                           a.nby, a.nbx, a.M, hist, order);
        int workers = n_workers < total ? n_workers : total;
        if (eb) (void)hipEventRecord(eb, s);
        hipLaunchKernelGGL((raster_persistent_kernel<KB, EXACT, OPT>), dim3(workers), dim3(64), 0, s, a, order, hdr,
                           total);
        if (ee) (void)hipEventRecord(ee, s);
        return hipGetLastError();
    }
    dim3 grid(a.tiles_x, a.tiles_y, a.N);
    if (eb) (void)hipEventRecord(eb, s);
    if (binned)
        hipLaunchKernelGGL((raster_tiles_kernel<KB, true, EXACT, OPT>), grid, dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((raster_tiles_kernel<KB, false, EXACT, OPT>), grid, dim3(64), 0, s, a);
    if (ee) (void)hipEventRecord(ee, s);
    return hipGetLastError();
}

hipError_t launch_fine(const FaceRec* recs, const int64_t* first, const int64_t* nf, const int* counts,
                       const int* lists, int64_t F, int N, int H, int W, int K, float blur, int opts, int bs, int M,
                       int sched,
                       int* order, int* hist, int* hdr, int n_workers, int32_t* p2f, float* zbuf, float* bary,
                       float* dists, hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    FineArgs a;
    a.recs = recs;
    a.first = first;
    a.nf = nf;
    a.counts = counts;
    a.lists = lists;
    a.F = F;
    a.N = N;
    a.H = H;
    a.W = W;
    a.K = K;
    a.blur = blur;
    a.opts = opts;
    a.bs = bs > 0 ? bs : kTile;
    a.nby = bs > 0 ? (H + bs - 1) / bs : 0;
    a.nbx = bs > 0 ? (W + bs - 1) / bs : 0;
    a.M = M;
    a.tiles_x = (W + kTile - 1) / kTile;
    a.tiles_y = (H + kTile - 1) / kTile;
    a.p2f = p2f;
    a.zbuf = zbuf;
    a.bary = bary;
    a.dists = dists;
    bool binned = bs > 0;
    // queue sizes are powers of two; K equal to one gets the compile-time-K
    // kernels, which store four slots at a time and so need 16-byte aligned
    // outputs
    const bool aligned = (((uintptr_t)p2f | (uintptr_t)zbuf | (uintptr_t)bary | (uintptr_t)dists) & 15) == 0;
#define RAST_FINE_BUCKET(KB)                                                                          \
    if (K <= KB) {                                                                                    \
        if (opt) return launch_fine_k<KB, false, true>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee); \
        if (K == KB && aligned)                                                                         \
            return launch_fine_k<KB, true, false>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee); \
        return launch_fine_k<KB, false, false>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee); \
    }
    // options that change barycentrics and depth take the runtime-K form with their per-pixel work
    const bool opt = (opts & (kOptPersp | kOptClip)) != 0;
    if (K <= 1 && opt) return launch_fine_k<1, true, true>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee);
    if (K <= 2 && opt) return launch_fine_k<2, true, true>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee);
    if (K <= 1) return launch_fine_k<1, true, false>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee);
    if (K <= 2) return launch_fine_k<2, true, false>(a, binned, sched, order, hist, hdr, n_workers, s, eb, ee);
    RAST_FINE_BUCKET(4)
    RAST_FINE_BUCKET(8)
    RAST_FINE_BUCKET(16)
    RAST_FINE_BUCKET(32)
    RAST_FINE_BUCKET(64)
#undef RAST_FINE_BUCKET
    return hipErrorInvalidValue;
}

}  // namespace rast
