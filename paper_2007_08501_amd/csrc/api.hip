// api.hip -- the library's C ABI (declared in include/rast.h): argument
// validation on the host, workspace layout, and the launch sequence of each
// entry point on the caller's stream.  No allocation, no synchronisation
// (except rast_query_status).
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <atomic>

#include <hip/hip_runtime.h>

#include "../../include/rast.h"
#include "device.hpp"
#include "launch.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t hdr, recs, counts, lists, order, hist, partial, big, total;
    int nby, nbx, tiles_x, tiles_y;
    int64_t nbins;
};

// Workspace layout; returns false if a size does not fit in size_t.
bool make_layout(int N, int H, int W, int64_t F, int bs, int M, Layout* L) {
    const size_t big = (size_t)1 << 62;
    size_t off = 0;
    L->hdr = off;
    off += kAlign;
    L->recs = off;
    if ((size_t)F > big / sizeof(rast::FaceRec)) return false;
    off = align_up(off + (size_t)F * sizeof(rast::FaceRec));
    L->tiles_x = (W + rast::kTile - 1) / rast::kTile;
    L->tiles_y = (H + rast::kTile - 1) / rast::kTile;
    L->nby = L->nbx = 0;
    L->nbins = 0;
    L->counts = L->lists = L->order = L->hist = off;
    if (bs > 0) {
        L->nby = (H + bs - 1) / bs;
        L->nbx = (W + bs - 1) / bs;
        L->nbins = (int64_t)N * L->nby * L->nbx;
        L->counts = off;
        off = align_up(off + (size_t)L->nbins * 4);
        L->lists = off;
        size_t ls = (size_t)L->nbins * (size_t)(M > 0 ? M : 0);
        if (ls > big / 4) return false;
        off = align_up(off + ls * 4);
        L->order = off;
        off = align_up(off + (size_t)N * L->tiles_x * L->tiles_y * 4);
        L->hist = off;
        off = align_up(off + 64 * 4);
    }
    // backward only: per-face partial sums, one per bin of the face's range
    // (F x 4 x 9 floats), and the list of large faces (F ints)
    L->partial = off;
    if ((size_t)F > big / 144) return false;
    off = align_up(off + (size_t)F * 144);
    L->big = off;
    off = align_up(off + (size_t)F * 4);
    L->total = off;
    return true;
}

bool bad_dims(int N, int H, int W, int K) {
    if (N < 1 || H < 1 || W < 1) return true;
    if (K < 1 || K > RAST_KMAX) return true;
    // keep N*H*W*K*3 well inside int64 and every per-image pixel index in int32
    if ((int64_t)H * W > ((int64_t)1 << 30)) return true;
    if ((int64_t)N * H * W * K > ((int64_t)1 << 40)) return true;
    // the fine pass addresses a tile's fragments with 32-bit offsets (8 rows of 3*K floats per pixel)
    if ((int64_t)W * K * 3 * RAST_TILE > INT32_MAX) return true;
    return false;
}

int n_workers_for_current_device() {
    static int cached[kMaxDevices] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 1024;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus * 32;
    }
    return cached[dev];
}

inline int hip_rc(hipError_t e) { return e == hipSuccess ? RAST_OK : RAST_EHIP; }

// Instrumentation events of the calling host thread (rast_set_kernel_events).
struct KernelEvents {
    hipEvent_t begin[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t end[4] = {nullptr, nullptr, nullptr, nullptr};
};
thread_local KernelEvents tl_events;

}  // namespace

// The scratch of rasterize_meshes_fwd_static: one per GPU, for the life of the
// process.  In host code its name is only a stand-in: kernels get the
// device address from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) unsigned char scratch[RAST_STATIC_SCRATCH_BYTES];

namespace {
std::atomic<void*> g_scratch_addr[kMaxDevices];

// Device address of the current device's scratch (looked up on the first
// call on that device); nullptr if the device or the lookup fails.
void* static_scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    void* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || q == nullptr) return nullptr;
        g_scratch_addr[dev].store(q, std::memory_order_release);
        p = q;
    }
    return p;
}
}  // namespace

static rast::BinSig bin_signature(int64_t F, int N, int H, int W, int bs, int M, float blur, int opts) {
    rast::BinSig g;
    uint32_t bb;
    memcpy(&bb, &blur, sizeof(bb));
    // the options change which faces count: they share the marker word
    const int w[rast::kSigWords] = {rast::kSigMarker ^ opts, (int)F, N, H, W, bs, M, (int)bb};
    for (int i = 0; i < rast::kSigWords; ++i) g.w[i] = w[i];
    return g;
}

// The forward on a caller workspace or the static scratch.  status_out
// (device, nullable) receives the device status at the end of the call.
static int fwd_impl(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                    const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh, int N, int H, int W,
                    float blur_radius, int faces_per_pixel, int bin_size, int max_faces_per_bin, int sched,
                    int options, int32_t* pix_to_face, float* zbuf, float* bary, float* dists, void* workspace,
                    size_t workspace_bytes, bool static_scratch, int32_t* status_out, void* stream) {
    if (bad_dims(N, H, W, faces_per_pixel)) return RAST_EINVAL;
    if ((options & ~rast::kOptMask) != 0) return RAST_EINVAL;
    if (V < 0 || V > INT32_MAX || F < 0 || F > INT32_MAX) return RAST_EINVAL;
    if ((V > 0 && verts_packed == nullptr) || (F > 0 && faces_packed == nullptr)) return RAST_EINVAL;
    if (mesh_to_face_first_idx == nullptr || num_faces_per_mesh == nullptr) return RAST_EINVAL;
    if (pix_to_face == nullptr || zbuf == nullptr || bary == nullptr || dists == nullptr) return RAST_EINVAL;
    if (!(blur_radius >= 0.0f) || !isfinite(blur_radius)) return RAST_EINVAL;
    if (bin_size < 0 || bin_size > RAST_MAX_BIN || (bin_size % RAST_TILE) != 0) return RAST_EINVAL;
    if (bin_size > 0 && max_faces_per_bin < 1) return RAST_EINVAL;
    if (sched != RAST_SCHED_GRID && sched != RAST_SCHED_PERSISTENT) return RAST_EINVAL;
    Layout L;
    if (!make_layout(N, H, W, F, bin_size, max_faces_per_bin, &L)) return RAST_EINVAL;
    if (static_scratch) {
        if (L.total > RAST_STATIC_SCRATCH_BYTES) return RAST_ESCRATCH;
        workspace = static_scratch_ptr();
        workspace_bytes = RAST_STATIC_SCRATCH_BYTES;
        if (workspace == nullptr) return RAST_EHIP;
    }
    if (workspace == nullptr || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
        return RAST_EWORKSPACE;

    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    int* hdr = (int*)(ws + L.hdr);
    rast::FaceRec* recs = (rast::FaceRec*)(ws + L.recs);
    int n_workers = (sched == RAST_SCHED_PERSISTENT) ? n_workers_for_current_device() : 0;

    // the header carries this call's binning signature for a backward that reuses the bins
    hipError_t e = rast::launch_header_init(
        hdr, bin_signature(F, N, H, W, bin_size, bin_size > 0 ? max_faces_per_bin : 0, blur_radius, options), s);
    if (e != hipSuccess) return RAST_EHIP;
    e = rast::launch_face_setup(verts_packed, V, faces_packed, F, mesh_to_face_first_idx, num_faces_per_mesh, N,
                                sqrtf(blur_radius), options, recs, hdr, s);
    if (e != hipSuccess) return RAST_EHIP;
    int* counts = nullptr;
    int* lists = nullptr;
    if (bin_size > 0) {
        counts = (int*)(ws + L.counts);
        lists = (int*)(ws + L.lists);
        e = rast::launch_binning(recs, F, N, H, W, bin_size, max_faces_per_bin, counts, lists, hdr, s);
        if (e != hipSuccess) return RAST_EHIP;
    }
    e = rast::launch_fine(recs, mesh_to_face_first_idx, num_faces_per_mesh, counts, lists, F, N, H, W,
                          faces_per_pixel, blur_radius, options, bin_size, max_faces_per_bin, sched,
                          (int*)(ws + L.order),
                          (int*)(ws + L.hist), hdr, n_workers, pix_to_face, zbuf, bary, dists, s,
                          tl_events.begin[RAST_KERNEL_FINE], tl_events.end[RAST_KERNEL_FINE]);
    if (e != hipSuccess) return RAST_EHIP;
    if (status_out != nullptr) e = rast::launch_status_out(hdr, status_out, s);
    return hip_rc(e);
}

extern "C" {

int rast_workspace_size(int N, int H, int W, int64_t F, int bin_size, int max_faces_per_bin, size_t* bytes_out) {
    if (bytes_out == nullptr) return RAST_EINVAL;
    if (N < 1 || H < 1 || W < 1 || F < 0 || F > INT32_MAX) return RAST_EINVAL;
    if (bin_size < 0 || bin_size > RAST_MAX_BIN || (bin_size % RAST_TILE) != 0) return RAST_EINVAL;
    if (bin_size > 0 && max_faces_per_bin < 1) return RAST_EINVAL;
    Layout L;
    if (!make_layout(N, H, W, F, bin_size, max_faces_per_bin, &L)) return RAST_EINVAL;
    *bytes_out = L.total;
    return RAST_OK;
}

int rasterize_meshes_fwd(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                         const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh, int N, int H,
                         int W, float blur_radius, int faces_per_pixel, int bin_size, int max_faces_per_bin,
                         int sched, int options, int32_t* pix_to_face, float* zbuf, float* bary, float* dists,
                         void* workspace, size_t workspace_bytes, void* stream) {
    return fwd_impl(verts_packed, V, faces_packed, F, mesh_to_face_first_idx, num_faces_per_mesh, N, H, W,
                    blur_radius, faces_per_pixel, bin_size, max_faces_per_bin, sched, options, pix_to_face, zbuf,
                    bary, dists, workspace, workspace_bytes, false, nullptr, stream);
}

int rasterize_meshes_fwd_static(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                                const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh, int N,
                                int H, int W, float blur_radius, int faces_per_pixel, int bin_size,
                                int max_faces_per_bin, int sched, int options, int32_t* pix_to_face, float* zbuf,
                                float* bary, float* dists, int32_t* status_out, void* stream) {
    return fwd_impl(verts_packed, V, faces_packed, F, mesh_to_face_first_idx, num_faces_per_mesh, N, H, W,
                    blur_radius, faces_per_pixel, bin_size, max_faces_per_bin, sched, options, pix_to_face, zbuf,
                    bary, dists, nullptr, 0, true, status_out, stream);
}

int rasterize_meshes_bwd(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                         const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh, int N, int H,
                         int W, float blur_radius, int faces_per_pixel, int bin_size, int max_faces_per_bin,
                         int flags, const int32_t* pix_to_face, const float* grad_zbuf, const float* grad_bary,
                         const float* grad_dists, float* grad_verts, void* workspace, size_t workspace_bytes,
                         void* stream) {
    if (bad_dims(N, H, W, faces_per_pixel)) return RAST_EINVAL;
    if (V < 0 || V > INT32_MAX || F < 0 || F > INT32_MAX) return RAST_EINVAL;
    if ((V > 0 && (verts_packed == nullptr || grad_verts == nullptr)) || (F > 0 && faces_packed == nullptr))
        return RAST_EINVAL;
    if (mesh_to_face_first_idx == nullptr || num_faces_per_mesh == nullptr) return RAST_EINVAL;
    if (pix_to_face == nullptr) return RAST_EINVAL;
    if ((flags & ~(RAST_BWD_REUSE_FORWARD | rast::kOptMask)) != 0) return RAST_EINVAL;
    const int options = flags & rast::kOptMask;
    if (!(blur_radius >= 0.0f) || !isfinite(blur_radius)) return RAST_EINVAL;
    if (bin_size < 0 || bin_size > RAST_MAX_BIN || (bin_size % RAST_TILE) != 0) return RAST_EINVAL;
    if (bin_size > 0 && max_faces_per_bin < 1) return RAST_EINVAL;
    Layout L;
    if (!make_layout(N, H, W, F, bin_size, max_faces_per_bin, &L)) return RAST_EINVAL;
    if (workspace == nullptr || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
        return RAST_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (V == 0) return RAST_OK;
    char* ws = (char*)workspace;
    return hip_rc(rast::launch_backward(
        verts_packed, V, faces_packed, F, mesh_to_face_first_idx, num_faces_per_mesh, N, H, W, faces_per_pixel,
        blur_radius, options, bin_size, max_faces_per_bin, pix_to_face, grad_zbuf, grad_bary, grad_dists, grad_verts,
        (int*)(ws + L.hdr), (rast::FaceRec*)(ws + L.recs), (int*)(ws + L.counts), (int*)(ws + L.lists),
        (float*)(ws + L.partial), (int*)(ws + L.big), (flags & RAST_BWD_REUSE_FORWARD) != 0,
        bin_signature(F, N, H, W, bin_size, bin_size > 0 ? max_faces_per_bin : 0, blur_radius, options), s,
        tl_events.begin[RAST_KERNEL_BWD], tl_events.end[RAST_KERNEL_BWD]));
}

int rast_set_kernel_events(int kernel, void* begin, void* end) {
    if (kernel < RAST_KERNEL_FINE || kernel > RAST_KERNEL_POINTS_BWD) return RAST_EINVAL;
    if ((begin == nullptr) != (end == nullptr)) return RAST_EINVAL;
    tl_events.begin[kernel] = (hipEvent_t)begin;
    tl_events.end[kernel] = (hipEvent_t)end;
    return RAST_OK;
}

int rast_bin_count(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                   const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh, int N, int H, int W,
                   float blur_radius, int bin_size, void* workspace, size_t workspace_bytes, void* stream) {
    if (N < 1 || H < 1 || W < 1) return RAST_EINVAL;
    if (V < 0 || V > INT32_MAX || F < 0 || F > INT32_MAX) return RAST_EINVAL;
    if ((V > 0 && verts_packed == nullptr) || (F > 0 && faces_packed == nullptr)) return RAST_EINVAL;
    if (mesh_to_face_first_idx == nullptr || num_faces_per_mesh == nullptr) return RAST_EINVAL;
    if (!(blur_radius >= 0.0f) || !isfinite(blur_radius)) return RAST_EINVAL;
    if (bin_size < RAST_TILE || bin_size > RAST_MAX_BIN || (bin_size % RAST_TILE) != 0) return RAST_EINVAL;
    Layout L;
    if (!make_layout(N, H, W, F, bin_size, 1, &L)) return RAST_EINVAL;
    if (workspace == nullptr || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
        return RAST_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    int* hdr = (int*)(ws + L.hdr);
    rast::FaceRec* recs = (rast::FaceRec*)(ws + L.recs);
    hipError_t e = rast::launch_fill_i32(hdr, rast::kHdrWords, 0, s);
    if (e != hipSuccess) return RAST_EHIP;
    e = rast::launch_face_setup(verts_packed, V, faces_packed, F, mesh_to_face_first_idx, num_faces_per_mesh, N,
                                sqrtf(blur_radius), 0, recs, hdr, s);
    if (e != hipSuccess) return RAST_EHIP;
    // M = 0: count only, no list writes
    return hip_rc(rast::launch_binning(recs, F, N, H, W, bin_size, 0, (int*)(ws + L.counts), nullptr, hdr, s));
}

int rast_query_status(const void* workspace, int* status, int* max_bin_count, void* stream) {
    if (workspace == nullptr || status == nullptr) return RAST_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int h[2] = {0, 0};
    if (hipMemcpyAsync(h, workspace, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return RAST_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RAST_EHIP;
    int st = RAST_OK;
    if (h[0] & rast::kStatMesh)
        st = RAST_EMESH;
    else if (h[0] & rast::kStatReuse)
        st = RAST_EREUSE;
    else if (h[0] & rast::kStatOverflow)
        st = RAST_EOVERFLOW;
    *status = st;
    if (max_bin_count) *max_bin_count = h[1];
    return RAST_OK;
}

const char* rast_status_string(int status) {
    switch (status) {
        case RAST_OK: return "ok";
        case RAST_EINVAL: return "invalid argument";
        case RAST_EWORKSPACE: return "workspace missing, too small or misaligned";
        case RAST_EHIP: return "HIP launch failed";
        case RAST_EOVERFLOW: return "a bin received more faces than max_faces_per_bin";
        case RAST_EMESH: return "mesh face ranges or vertex ids out of range";
        case RAST_EREUSE: return "the workspace does not hold the bins of a matching forward";
        case RAST_ESCRATCH: return "the problem needs more than the static scratch (RAST_STATIC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

int silhouette_blend_fwd(const int32_t* pix_to_face, const float* dists, int64_t P, int K, float sigma, float* alpha,
                         void* stream) {
    if (P < 0 || K < 1 || K > RAST_KMAX || !(sigma > 0.0f) || !isfinite(sigma)) return RAST_EINVAL;
    if (P > 0 && (pix_to_face == nullptr || dists == nullptr || alpha == nullptr)) return RAST_EINVAL;
    return hip_rc(rast::launch_blend_fwd(pix_to_face, dists, P, K, sigma, alpha, (hipStream_t)stream));
}

int silhouette_blend_bwd(const int32_t* pix_to_face, const float* dists, const float* grad_alpha, int64_t P, int K,
                         float sigma, float* grad_dists, void* stream) {
    if (P < 0 || K < 1 || K > RAST_KMAX || !(sigma > 0.0f) || !isfinite(sigma)) return RAST_EINVAL;
    if (P > 0 && (pix_to_face == nullptr || dists == nullptr || grad_alpha == nullptr || grad_dists == nullptr))
        return RAST_EINVAL;
    return hip_rc(rast::launch_blend_bwd(pix_to_face, dists, grad_alpha, P, K, sigma, grad_dists,
                                         (hipStream_t)stream));
}

static bool bad_softmax(int64_t P, int K, int C, float sigma, float gamma, float znear, float zfar) {
    if (P < 0 || K < 1 || K > RAST_KMAX || C < 1 || C > RAST_SOFTMAX_CMAX) return true;
    if (!(sigma > 0.0f) || !isfinite(sigma) || !(gamma > 0.0f) || !isfinite(gamma)) return true;
    if (!isfinite(znear) || !isfinite(zfar) || !(zfar > znear)) return true;
    if (!isfinite((float)(1.0 / (((double)zfar - (double)znear) * (double)gamma)))) return true;
    return false;
}

int softmax_blend_fwd(const int32_t* pix_to_face, const float* zbuf, const float* dists, const float* colors,
                      int64_t P, int K, int C, float sigma, float gamma, float znear, float zfar, float* image,
                      void* stream) {
    if (bad_softmax(P, K, C, sigma, gamma, znear, zfar)) return RAST_EINVAL;
    if (P > 0 && (pix_to_face == nullptr || zbuf == nullptr || dists == nullptr || colors == nullptr ||
                  image == nullptr))
        return RAST_EINVAL;
    return hip_rc(rast::launch_softmax_fwd(pix_to_face, zbuf, dists, colors, P, K, C, sigma, gamma, znear, zfar, image,
                                           (hipStream_t)stream));
}

int softmax_blend_bwd(const int32_t* pix_to_face, const float* zbuf, const float* dists, const float* colors,
                      int64_t P, int K, int C, float sigma, float gamma, float znear, float zfar,
                      const float* grad_image, float* grad_zbuf, float* grad_dists, float* grad_colors, void* stream) {
    if (bad_softmax(P, K, C, sigma, gamma, znear, zfar)) return RAST_EINVAL;
    if (P > 0 && (pix_to_face == nullptr || zbuf == nullptr || dists == nullptr || colors == nullptr ||
                  grad_image == nullptr))
        return RAST_EINVAL;
    return hip_rc(rast::launch_softmax_bwd(pix_to_face, zbuf, dists, colors, P, K, C, sigma, gamma, znear, zfar,
                                           grad_image, grad_zbuf, grad_dists, grad_colors, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// Point clouds
// ---------------------------------------------------------------------------
namespace {

struct PtLayout {
    size_t hdr, start, bsum, home, rank, sorted, order, ohist, total;
};

bool make_pt_layout(int N, int H, int W, int64_t P, PtLayout* L) {
    const int64_t T = (int64_t)N * ((H + rast::kTile - 1) / rast::kTile) * ((W + rast::kTile - 1) / rast::kTile);
    if (T + 1 > INT32_MAX || P < 0 || P > RAST_POINTS_MAX) return false;
    size_t off = 0;
    L->hdr = off;
    off += kAlign;
    L->start = off;
    off = align_up(off + (size_t)(T + 1) * 4);
    L->bsum = off;
    off = align_up(off + (size_t)(rast::pt_scan_blocks(T) + 1) * 4);
    L->home = off;
    off = align_up(off + (size_t)P * 4);
    L->rank = off;
    off = align_up(off + (size_t)P * 4);
    L->sorted = off;
    off = align_up(off + (size_t)P * 16);
    L->order = off;
    off = align_up(off + (size_t)T * 4);
    L->ohist = off;
    off = align_up(off + 64 * 4);
    L->total = off;
    return true;
}

bool bad_points(int N, int H, int W, int K, int64_t P, float radius) {
    if (bad_dims(N, H, W, K)) return true;
    // pixel ranges of discs are conservative to well under 0.01 pixel up to this size
    if (H > RAST_POINTS_MAX_SIDE || W > RAST_POINTS_MAX_SIDE) return true;
    if (P < 0 || P > RAST_POINTS_MAX) return true;
    if (!isfinite(radius) || !(radius >= 0.0f) || radius > RAST_POINTS_MAX_RADIUS) return true;
    return false;
}

rast::BinSig pt_signature(int64_t P, int N, int H, int W, float radius) {
    rast::BinSig g;
    uint32_t rb;
    memcpy(&rb, &radius, sizeof(rb));
    const int w[rast::kSigWords] = {rast::kPtSigMarker, (int)P, N, H, W, (int)rb, 0, 0};
    for (int i = 0; i < rast::kSigWords; ++i) g.w[i] = w[i];
    return g;
}

}  // namespace

int rast_points_workspace_size(int N, int H, int W, int64_t P, size_t* bytes_out) {
    if (bytes_out == nullptr || N < 1 || H < 1 || W < 1) return RAST_EINVAL;
    PtLayout L;
    if (!make_pt_layout(N, H, W, P, &L)) return RAST_EINVAL;
    *bytes_out = L.total;
    return RAST_OK;
}

int rasterize_points_fwd(const float* points, int64_t P, const int64_t* cloud_to_first_idx,
                         const int64_t* num_points_per_cloud, int N, int H, int W, float radius, int points_per_pixel,
                         int32_t* idx, float* zbuf, float* dists, void* workspace, size_t workspace_bytes,
                         void* stream) {
    if (bad_points(N, H, W, points_per_pixel, P, radius)) return RAST_EINVAL;
    if ((P > 0 && points == nullptr) || cloud_to_first_idx == nullptr || num_points_per_cloud == nullptr)
        return RAST_EINVAL;
    if (idx == nullptr || zbuf == nullptr || dists == nullptr) return RAST_EINVAL;
    PtLayout L;
    if (!make_pt_layout(N, H, W, P, &L)) return RAST_EINVAL;
    if (workspace == nullptr || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
        return RAST_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    int* hdr = (int*)(ws + L.hdr);
    if (rast::launch_header_init(hdr, pt_signature(P, N, H, W, radius), s) != hipSuccess) return RAST_EHIP;
    return hip_rc(rast::launch_points_fwd(points, P, cloud_to_first_idx, num_points_per_cloud, N, H, W, radius,
                                          points_per_pixel, hdr, (int*)(ws + L.start), (int*)(ws + L.bsum),
                                          (int*)(ws + L.home), (int*)(ws + L.rank), (float4*)(ws + L.sorted),
                                          (int*)(ws + L.order), (int*)(ws + L.ohist), idx, zbuf, dists, s,
                                          tl_events.begin[RAST_KERNEL_POINTS_FINE],
                                          tl_events.end[RAST_KERNEL_POINTS_FINE]));
}

int rasterize_points_bwd(const float* points, int64_t P, const int64_t* cloud_to_first_idx,
                         const int64_t* num_points_per_cloud, int N, int H, int W, float radius, int points_per_pixel,
                         int flags, const int32_t* idx, const float* grad_zbuf, const float* grad_dists,
                         float* grad_points, void* workspace, size_t workspace_bytes, void* stream) {
    if (bad_points(N, H, W, points_per_pixel, P, radius)) return RAST_EINVAL;
    if ((P > 0 && (points == nullptr || grad_points == nullptr)) || cloud_to_first_idx == nullptr ||
        num_points_per_cloud == nullptr || idx == nullptr)
        return RAST_EINVAL;
    if ((flags & ~RAST_BWD_REUSE_FORWARD) != 0) return RAST_EINVAL;
    PtLayout L;
    if (!make_pt_layout(N, H, W, P, &L)) return RAST_EINVAL;
    if (workspace == nullptr || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total)
        return RAST_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    return hip_rc(rast::launch_points_bwd(
        points, P, cloud_to_first_idx, num_points_per_cloud, N, H, W, radius, points_per_pixel, idx, grad_zbuf,
        grad_dists, grad_points, (int*)(ws + L.hdr), (int*)(ws + L.start), (int*)(ws + L.bsum), (int*)(ws + L.home),
        (int*)(ws + L.rank), (float4*)(ws + L.sorted), (int*)(ws + L.order), (int*)(ws + L.ohist),
        n_workers_for_current_device() / 32, (flags & RAST_BWD_REUSE_FORWARD) != 0,
        pt_signature(P, N, H, W, radius), s, tl_events.begin[RAST_KERNEL_POINTS_BWD],
        tl_events.end[RAST_KERNEL_POINTS_BWD]));
}

static bool bad_composite(int64_t P, int64_t npix, int K, int D, int mode, float radius) {
    if (P < 0 || P > INT32_MAX || npix < 0 || K < 1 || K > RAST_KMAX || D < 1 || D > RAST_COMPOSITE_DMAX) return true;
    if ((mode & ~(RAST_COMPOSITE_NORM | RAST_COMPOSITE_FROM_DISTS)) != 0) return true;
    if (npix > ((int64_t)1 << 40) / K) return true;
    if (mode & RAST_COMPOSITE_FROM_DISTS) {
        if (!isfinite(radius) || !(radius > 0.0f)) return true;
        if (!isfinite((float)(1.0 / ((double)radius * (double)radius)))) return true;
    }
    return false;
}

int points_composite_fwd(const int32_t* idx, const float* weights, const float* features, int64_t P, int64_t npix,
                         int K, int D, int mode, float radius, float* image, void* stream) {
    if (bad_composite(P, npix, K, D, mode, radius)) return RAST_EINVAL;
    if (npix > 0 && (idx == nullptr || weights == nullptr || image == nullptr)) return RAST_EINVAL;
    return hip_rc(rast::launch_composite_fwd(idx, weights, features, P, npix, K, D, mode, radius, image,
                                             (hipStream_t)stream));
}

int points_composite_bwd(const int32_t* idx, const float* weights, const float* features, int64_t P, int64_t npix,
                         int K, int D, int mode, float radius, const float* grad_image, float* grad_weights,
                         float* grad_features, void* stream) {
    if (bad_composite(P, npix, K, D, mode, radius)) return RAST_EINVAL;
    if (npix > 0 && (idx == nullptr || weights == nullptr || grad_image == nullptr || grad_weights == nullptr))
        return RAST_EINVAL;
    if (features == nullptr && grad_features != nullptr) return RAST_EINVAL;
    return hip_rc(rast::launch_composite_bwd(idx, weights, features, P, npix, K, D, mode, radius, grad_image,
                                             grad_weights, grad_features, (hipStream_t)stream));
}

}  // extern "C"
