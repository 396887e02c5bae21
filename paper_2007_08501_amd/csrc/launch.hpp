// launch.hpp -- host-side launchers of the rasterizer kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace rast {

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_header_init(int* hdr, const BinSig& sig, hipStream_t s);
// out[0] = the header's device status as a rast_status code, out[1] = its largest bin count
hipError_t launch_status_out(const int* hdr, int32_t* out, hipStream_t s);

hipError_t launch_face_setup(const float* verts, int64_t V, const int32_t* faces, int64_t F, const int64_t* first,
                             const int64_t* nf, int N, float rb, int opts, FaceRec* recs, int* hdr, hipStream_t s);

hipError_t launch_binning(const FaceRec* recs, int64_t F, int N, int H, int W, int bs, int M, int* counts, int* lists,
                          int* hdr, hipStream_t s);

hipError_t launch_fine(const FaceRec* recs, const int64_t* first, const int64_t* nf, const int* counts,
                       const int* lists, int64_t F, int N, int H, int W, int K, float blur, int opts, int bs, int M,
                       int sched,
                       int* order, int* hist, int* hdr, int n_workers, int32_t* p2f, float* zbuf, float* bary,
                       float* dists, hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end);

hipError_t launch_backward(const float* verts, int64_t V, const int32_t* faces, int64_t F, const int64_t* first,
                           const int64_t* nf, int N, int H, int W, int K, float blur, int opts, int bs, int M,
                           const int32_t* p2f, const float* gz, const float* gb, const float* gd, float* grad,
                           int* hdr, FaceRec* recs, int* counts, int* lists, float* partial, int* big,
                           bool reuse, const BinSig& sig, hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end);

hipError_t launch_blend_fwd(const int32_t* p2f, const float* d, int64_t P, int K, float sigma, float* alpha,
                            hipStream_t s);
hipError_t launch_blend_bwd(const int32_t* p2f, const float* d, const float* ga, int64_t P, int K, float sigma,
                            float* gd, hipStream_t s);
hipError_t launch_softmax_fwd(const int32_t* p2f, const float* z, const float* d, const float* col, int64_t P, int K,
                              int C, float sigma, float gamma, float znear, float zfar, float* img, hipStream_t s);
hipError_t launch_softmax_bwd(const int32_t* p2f, const float* z, const float* d, const float* col, int64_t P, int K,
                              int C, float sigma, float gamma, float znear, float zfar, const float* gimg, float* gz,
                              float* gd, float* gc, hipStream_t s);


// point clouds (kernels_points.hip)
int64_t pt_scan_blocks(int64_t T);
hipError_t launch_points_fwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, int* hdr, int* start, int* bsum, int* home, int* rank,
                             float4* sorted, int* order, int* ohist, int32_t* idx, float* zbuf, float* dists,
                             hipStream_t s, hipEvent_t eb, hipEvent_t ee);
hipError_t launch_points_bwd(const float* pts, int64_t P, const int64_t* first, const int64_t* np, int N, int H,
                             int W, float radius, int K, const int32_t* idx, const float* gz, const float* gd,
                             float* grad, int* hdr, int* start, int* bsum, int* home, int* rank, float4* sorted,
                             int* order, int* ohist, int n_cus, bool reuse, const BinSig& sig, hipStream_t s,
                             hipEvent_t eb, hipEvent_t ee);
hipError_t launch_composite_fwd(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K,
                                int D, int mode, float radius, float* img, hipStream_t s);
hipError_t launch_composite_bwd(const int32_t* idx, const float* w, const float* f, int64_t P, int64_t npix, int K,
                                int D, int mode, float radius, const float* gimg, float* gw, float* gf,
                                hipStream_t s);

}  // namespace rast
