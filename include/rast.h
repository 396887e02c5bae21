/*
 * rast.h -- C ABI of the MI355X (gfx950) batched differentiable mesh and point-cloud rasterizer.
 *
 * The operation (paper, Section 3.2, "Rasterizer"): for every pixel of every
 * image in a heterogeneous batch of triangle meshes, find the K faces nearest
 * along z among the faces that cover the pixel or lie within a blur radius of
 * it, and return "Fragment data" for them: face id, barycentric coordinates of
 * the pixel in the face, z, and the signed xy distance from the pixel to the
 * face.  The forward works in two passes, image tiles first and pixels second
 * (same section); the backward turns gradients of the fragments into gradients
 * of the vertex positions, re-using the stored face ids rather than searching
 * again (same section).  The silhouette blend of Algorithm 1 (same section) is
 * exported beside it.
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers to memory the caller owns.  The
 *    library never allocates, frees or synchronises inside these calls (except
 *    rast_query_status, which says so) and launches only on `stream` (a
 *    hipStream_t; NULL = the default stream), so the calls can be captured in a
 *    HIP graph.  Host-side validation happens before any launch.
 *  - Return value: RAST_OK (0) or a negative rast_status.  A negative return
 *    means nothing was launched, except RAST_EHIP (a launch itself failed).
 *  - Conditions only the device can see (a bin overflow, inconsistent mesh
 *    ranges) are written to a sticky status word inside the workspace and
 *    read back with rast_query_status; the outputs of such a call are invalid.
 *  - Calls that share a workspace must not overlap; calls with distinct
 *    workspaces may run concurrently.
 *
 * Geometry conventions:
 *  - verts_packed (V,3) float32, view space: x, y in normalised device
 *    coordinates, z the depth (faces count only where their interpolated
 *    z >= 0).  Pixel (r, c) of an H x W image has its centre at
 *    x = 1 - (2c+1)/W, y = 1 - (2r+1)/H (+x to the left, +y up, row 0 at the
 *    top).
 *  - faces_packed (F,3) int32: global (packed) vertex ids.
 *  - mesh n owns faces [mesh_to_face_first_idx[n], ... + num_faces_per_mesh[n])
 *    (int64, device); ranges must be ascending and non-overlapping.  Image n
 *    is rendered from mesh n only.
 *  - Barycentrics are raw screen-space ones (no clipping, no perspective
 *    correction); z is interpolated with them.  dists is the squared xy
 *    distance to the nearest point of the triangle boundary, negative when the
 *    pixel is strictly inside (all barycentrics > 0), positive otherwise.
 *    blur_radius is in the same squared-NDC units: an outside face counts iff
 *    its squared distance is < blur_radius.  Faces with abs(2 * signed area)
 *    < 1e-8 never count.
 *  - Slots are ordered by ascending z, ties by ascending face id.  Empty slots
 *    hold pix_to_face = -1 and -1 in zbuf, all three bary and dists.
 */
#ifndef RAST_H
#define RAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rast_status {
    RAST_OK = 0,
    RAST_EINVAL = -1,      /* an argument is out of range or a required pointer is NULL */
    RAST_EWORKSPACE = -2,  /* workspace NULL, too small or not 256-byte aligned */
    RAST_EHIP = -3,        /* a HIP launch failed */
    RAST_EOVERFLOW = -4,   /* device: a bin received more than max_faces_per_bin faces */
    RAST_EMESH = -5,       /* device: mesh face ranges out of [0, F) or not ascending */
    RAST_EREUSE = -6,      /* device: a backward asked to reuse bins that the workspace does not hold */
    RAST_ESCRATCH = -7,    /* rasterize_meshes_fwd_static: the problem needs more than RAST_STATIC_SCRATCH_BYTES */
};

#define RAST_KMAX 64     /* largest faces_per_pixel */
#define RAST_TILE 8      /* the forward's work unit is an 8x8 pixel tile */
#define RAST_MAX_BIN 512 /* largest bin_size */

/* Flags for rasterize_meshes_bwd. */
#define RAST_BWD_REUSE_FORWARD 1 /* take face records and bins from the forward's workspace */

/* Scheduling flags for rasterize_meshes_fwd. */
#define RAST_SCHED_GRID 0       /* one workgroup per tile, hardware dispatch order */
#define RAST_SCHED_PERSISTENT 1 /* device-sized grid pulling tiles, most-loaded bins first */

/*
 * Rasterizer options: the `options` word of rasterize_meshes_fwd, or-ed into
 * the `flags` word of rasterize_meshes_bwd (which must name the forward's).
 * The paper leaves them to the camera and shader (Section 3.2); they are
 * defined here as follows.
 *  - RAST_PERSPECTIVE_CORRECT: barycentrics corrected for perspective,
 *    w'_i = (w_i / z_i) / sum_j (w_j / z_j) with the vertex depths z_i; a face
 *    with a vertex at z <= 0 never counts, nor does a (pixel, face) pair whose
 *    sum_j (w_j / z_j) is not positive.
 *  - RAST_CLIP_BARYCENTRIC: barycentrics (after the correction) clipped,
 *    w''_i = max(w_i, 0) / sum_j max(w_j, 0): a pixel outside the face within
 *    the blur radius takes the nearest point of the face.
 *  - RAST_CULL_BACKFACES: a face whose doubled signed area E in the x-y NDC
 *    plane is positive never counts (E < 0 is anticlockwise as the image is
 *    displayed, +x pointing left).
 * With the correction or the clipping, bary holds the final barycentrics,
 * zbuf = sum_i w_i z_i with them, and the z >= 0 test and the slot order use
 * that z; "inside" and dists stay geometric (raw barycentrics, xy distance).
 */
#define RAST_PERSPECTIVE_CORRECT 0x100
#define RAST_CLIP_BARYCENTRIC 0x200
#define RAST_CULL_BACKFACES 0x400

/*
 * Bytes of workspace needed by rasterize_meshes_fwd / _bwd / rast_bin_count
 * for these sizes (one size serves all three).  bin_size 0 selects the single-pass form (every pixel
 * against every face of its mesh).  bin_size > 0 must be a multiple of
 * RAST_TILE, at most RAST_MAX_BIN; max_faces_per_bin (M) > 0 then sizes the
 * per-bin face lists (N * ceil(H/bs) * ceil(W/bs) * M int32).
 */
int rast_workspace_size(int N, int H, int W, int64_t F, int bin_size, int max_faces_per_bin,
                        size_t* bytes_out);

/*
 * Forward (paper, Section 3.2: two passes, tiles then pixels, per-pixel
 * K-nearest selection, Fragment outputs).
 *   verts_packed (V,3) f32, faces_packed (F,3) i32, mesh_to_face_first_idx (N) i64,
 *   num_faces_per_mesh (N) i64 -- inputs, see the conventions above.
 *   N, H, W > 0 with H*W <= 2^30 and 24*W*K < 2^31; blur_radius >= 0 (squared NDC);
 *   faces_per_pixel K in [1, RAST_KMAX];
 *   bin_size 0 or a multiple of RAST_TILE <= RAST_MAX_BIN; max_faces_per_bin > 0 if bin_size > 0;
 *   sched: RAST_SCHED_GRID or RAST_SCHED_PERSISTENT (ignored when bin_size == 0).
 *   options: 0 or an or of RAST_PERSPECTIVE_CORRECT, RAST_CLIP_BARYCENTRIC,
 *   RAST_CULL_BACKFACES (any other bit: RAST_EINVAL).
 *   Outputs, row-major, fully overwritten:
 *     pix_to_face (N,H,W,K) i32 packed face id or -1
 *     zbuf (N,H,W,K) f32, bary (N,H,W,K,3) f32, dists (N,H,W,K) f32
 *   workspace: device memory of at least rast_workspace_size() bytes, 256-byte aligned.
 * An overflowing bin makes the call's outputs invalid and sets RAST_EOVERFLOW
 * in the workspace status (it is never a silent truncation).
 */
int rasterize_meshes_fwd(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                         const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh,
                         int N, int H, int W, float blur_radius, int faces_per_pixel, int bin_size,
                         int max_faces_per_bin, int sched, int options, int32_t* pix_to_face, float* zbuf,
                         float* bary, float* dists, void* workspace, size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the forward
 * above with the library's own scratch array in place of a caller workspace.
 * Same arguments, outputs and results as rasterize_meshes_fwd, except:
 *   - no workspace: the face records, bins and status word live in one
 *     static device array of RAST_STATIC_SCRATCH_BYTES per GPU, held from
 *     the first call on that GPU until the process ends; a problem whose
 *     rast_workspace_size() exceeds it is refused with RAST_ESCRATCH before
 *     any launch.  Nothing is allocated (no hipMalloc, no allocating library
 *     call); the scratch keeps the last call's contents and every call clears
 *     what it needs.
 *   - status_out: device int32[2], written at the end of the call on the
 *     stream: [0] the device-detected status (RAST_OK, RAST_EOVERFLOW,
 *     RAST_EMESH), [1] the largest bin count seen.  NULL: not written.
 *   - calls that overlap on one GPU (other streams or host threads) share the
 *     array and race: serialise them.  The scratch holds no bins for
 *     rasterize_meshes_bwd to reuse (use the workspace forms for training).
 */
#define RAST_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int rasterize_meshes_fwd_static(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                                const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh,
                                int N, int H, int W, float blur_radius, int faces_per_pixel, int bin_size,
                                int max_faces_per_bin, int sched, int options, int32_t* pix_to_face, float* zbuf,
                                float* bary, float* dists, int32_t* status_out, void* stream);

/*
 * Backward (paper, Section 3.2: gradients with respect to the inputs, from the
 * stored face ids).  For L = <grad_zbuf, zbuf> + <grad_bary, bary> +
 * <grad_dists, dists> over the slots with pix_to_face >= 0, writes dL/dverts
 * into grad_verts (V,3) f32, which is overwritten.  Each slot's barycentrics,
 * z and nearest edge are recomputed from the vertices; the choice of faces is
 * held fixed.  grad_zbuf (N,H,W,K), grad_bary (N,H,W,K,3) and grad_dists
 * (N,H,W,K) may each be NULL (= zero).
 *   pix_to_face must come from rasterize_meshes_fwd with the same vertices,
 *   faces, mesh ranges, image size and blur_radius; bin_size and
 *   max_faces_per_bin are the forward's (bin_size 0: the backward walks each
 *   face's pixel box; > 0: it streams each bin's slots once, gathering the
 *   faces they name, with the forward's bins for crowded bins).  In the
 *   binned form a slot id outside [0, F), or naming a face that never counts
 *   or one of another image, contributes nothing.
 *   A bin overflow sets RAST_EOVERFLOW in the workspace status and leaves
 *   grad_verts incomplete.
 *   flags: the forward's options, or-ed with RAST_BWD_REUSE_FORWARD or not;
 *   the gradient then runs through the options' barycentrics and depth.
 *   With RAST_BWD_REUSE_FORWARD and
 *   bin_size > 0, `workspace` must be the one the forward that produced
 *   pix_to_face used, not used by any call since, and the vertices must not
 *   have changed: the backward then takes the forward's face records and bins
 *   (and keeps its status) instead of rebuilding them.  The forward stamps its
 *   face count, image size, bin size, capacity, blur radius and options into the
 *   workspace; if they differ from this call's, the status becomes RAST_EREUSE
 *   and grad_verts is left zero.  Changed vertex contents cannot be detected.
 *   With bin_size == 0 the flag has no effect.
 * The result accumulates with float atomics, so its last bits may differ
 * between runs.  workspace: at least rast_workspace_size(N, H, W, F,
 * bin_size, max_faces_per_bin) bytes.
 */
int rasterize_meshes_bwd(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                         const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh,
                         int N, int H, int W, float blur_radius, int faces_per_pixel, int bin_size,
                         int max_faces_per_bin, int flags, const int32_t* pix_to_face, const float* grad_zbuf,
                         const float* grad_bary, const float* grad_dists, float* grad_verts, void* workspace,
                         size_t workspace_bytes, void* stream);

/*
 * Coarse pass only, counting: fills the workspace status with the largest
 * number of faces any bin of this bin_size receives (read it with
 * rast_query_status).  Used to size max_faces_per_bin exactly (without
 * culling; with RAST_CULL_BACKFACES it is an upper bound).  Needs
 * rast_workspace_size(N, H, W, F, bin_size, 1) bytes.
 */
int rast_bin_count(const float* verts_packed, int64_t V, const int32_t* faces_packed, int64_t F,
                   const int64_t* mesh_to_face_first_idx, const int64_t* num_faces_per_mesh,
                   int N, int H, int W, float blur_radius, int bin_size,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * Synchronises `stream`, then reads the sticky status of the last call that
 * used this workspace: *status = RAST_OK, RAST_EOVERFLOW, RAST_EMESH or RAST_EREUSE;
 * *max_bin_count (may be NULL) = the largest bin count seen by the last
 * binned forward or rast_bin_count.
 */
int rast_query_status(const void* workspace, int* status, int* max_bin_count, void* stream);

/* Static text for a status code. */
const char* rast_status_string(int status);

/*
 * Instrumentation (not part of the method): on the calling host thread, make
 * every later rasterize_meshes_fwd (kernel = RAST_KERNEL_FINE) or
 * rasterize_meshes_bwd (kernel = RAST_KERNEL_BWD) call record `begin` and
 * `end` (hipEvent_t created by the caller) on its stream immediately before
 * and after the launch of its per-pixel kernel, so the caller can time that
 * kernel alone.  Pass NULL for both to switch it off.  Do not leave events set
 * while capturing a graph.  Returns RAST_EINVAL for an unknown kernel or a
 * single NULL.  The point-cloud entries take RAST_KERNEL_POINTS_FINE and
 * RAST_KERNEL_POINTS_BWD the same way.
 */
#define RAST_KERNEL_FINE 0
#define RAST_KERNEL_BWD 1
#define RAST_KERNEL_POINTS_FINE 2 /* rasterize_points_fwd: the per-tile pass */
#define RAST_KERNEL_POINTS_BWD 3  /* rasterize_points_bwd: the per-point gather */
int rast_set_kernel_events(int kernel, void* begin, void* end);

/*
 * Silhouette blend (paper, Section 3.2, Algorithm 1): per pixel,
 * prob_k = sigmoid(-dists_k / sigma) for slots with pix_to_face >= 0 (0 for
 * empty slots) and alpha = 1 - prod_k (1 - prob_k).
 *   pix_to_face, dists: (P,K) with P = N*H*W pixels; alpha: (P) f32 output.
 *   sigma > 0; K in [1, RAST_KMAX].
 */
int silhouette_blend_fwd(const int32_t* pix_to_face, const float* dists, int64_t P, int K, float sigma,
                         float* alpha, void* stream);

/*
 * Backward of silhouette_blend_fwd: grad_dists (P,K) = grad_alpha * d alpha / d dists,
 * d alpha / d dists_k = -(1/sigma) prob_k (1 - prob_k) prod_{j != k} (1 - prob_j),
 * formed with prefix and suffix products (no division), 0 for empty slots.
 * grad_dists is overwritten.
 */
int silhouette_blend_bwd(const int32_t* pix_to_face, const float* dists, const float* grad_alpha, int64_t P,
                         int K, float sigma, float* grad_dists, void* stream);

/*
 * Softmax blend (paper, Section 3.2, Algorithm 2) over P pixels of K slots
 * and C channels (C in [1, RAST_SOFTMAX_CMAX]):
 *   prob_k = sigmoid(-dists_k / sigma), zinv_k = (zfar - zbuf_k) / (zfar - znear),
 *   w_k = prob_k exp((zinv_k - max_j zinv_j) / gamma),
 *   image_c = sum_k w_k colors_kc / sum_k w_k.
 * Slots with pix_to_face == -1 take no part (no weight, no say in the max);
 * a pixel whose weights sum to 0 gets 0.
 *   pix_to_face (P,K) i32, zbuf (P,K) f32, dists (P,K) f32 -- Fragments;
 *   colors (P,K,C) f32 -- per-slot colours; image (P,C) f32, overwritten.
 *   sigma > 0, gamma > 0, zfar > znear, all finite.
 */
#define RAST_SOFTMAX_CMAX 8
int softmax_blend_fwd(const int32_t* pix_to_face, const float* zbuf, const float* dists, const float* colors,
                      int64_t P, int K, int C, float sigma, float gamma, float znear, float zfar, float* image,
                      void* stream);

/*
 * Backward of softmax_blend_fwd for L = <grad_image, image>.  With
 * G_k = sum_c grad_image_c (colors_kc - image_c) / sum_j w_j:
 *   grad_dists_k = -G_k w_k (1 - prob_k) / sigma,
 *   grad_zbuf_k = -G_k w_k / (gamma (zfar - znear)),
 *   grad_colors_kc = grad_image_c w_k / sum_j w_j;
 * 0 for empty slots and for pixels whose weights sum to 0.  Each of
 * grad_zbuf (P,K), grad_dists (P,K), grad_colors (P,K,C) may be NULL (not
 * computed); the others are overwritten.
 */
int softmax_blend_bwd(const int32_t* pix_to_face, const float* zbuf, const float* dists, const float* colors,
                      int64_t P, int K, int C, float sigma, float gamma, float znear, float zfar,
                      const float* grad_image, float* grad_zbuf, float* grad_dists, float* grad_colors, void* stream);

/* ==========================================================================
 * Point clouds (paper, Section 3.3, "Differentiable point cloud renderer").
 *
 * Every point is splatted to a disc of radius `radius` (NDC units) in screen
 * space.  For every pixel of image n the rasterizer returns the K points of
 * cloud n nearest along z whose discs cover the pixel centre, with their z
 * and their squared xy distance to the centre; compositing then blends the
 * points' features by Alpha compositing or by a normalised weighted sum.
 *
 *  - points (P,3) float32: x, y in NDC (pixel centres as for meshes), z the
 *    depth.  Cloud n owns points [cloud_to_first_idx[n], ... +
 *    num_points_per_cloud[n]) (int64, device; ascending, non-overlapping,
 *    inside [0, P]; a violation is reported as RAST_EMESH by
 *    rast_query_status).  Points outside every cloud are ignored.
 *  - A point covers a pixel iff its z >= 0 and (x - px)^2 + (y - py)^2 <
 *    radius^2, the squared distance evaluated in FP64 from the float32
 *    coordinates and the FP64 pixel centre as (dx*dx) + (dy*dy), with no
 *    fused operations: the decision is the same bit for bit as that plain
 *    evaluation.
 *  - Slots are ordered by ascending z, ties by ascending point index.  Empty
 *    slots hold idx = -1, zbuf = -1, dists = -1.  dists is the FP64 squared
 *    distance rounded to float32.
 *  - Limits: P <= RAST_POINTS_MAX, H and W <= RAST_POINTS_MAX_SIDE,
 *    0 <= radius <= RAST_POINTS_MAX_RADIUS, K in [1, RAST_KMAX].
 * ========================================================================== */
#define RAST_POINTS_MAX ((int64_t)1 << 30)
#define RAST_POINTS_MAX_SIDE 16384
#define RAST_POINTS_MAX_RADIUS 2.0f

/*
 * Bytes of workspace for rasterize_points_fwd / _bwd with these sizes: a
 * header, per-tile point counts and starts, and the points sorted by home
 * tile (16 bytes per point), about 24 bytes per point in all.
 */
int rast_points_workspace_size(int N, int H, int W, int64_t P, size_t* bytes_out);

/*
 * Forward.  Outputs idx (N,H,W,K) int32, zbuf and dists (N,H,W,K) float32,
 * all overwritten (K = points_per_pixel).  The workspace keeps the sorted
 * points for a backward with RAST_BWD_REUSE_FORWARD.
 * Errors: RAST_EINVAL (sizes, limits, NULL pointers), RAST_EWORKSPACE,
 * RAST_EHIP; device-side RAST_EMESH via rast_query_status.
 */
int rasterize_points_fwd(const float* points, int64_t P, const int64_t* cloud_to_first_idx,
                         const int64_t* num_points_per_cloud, int N, int H, int W, float radius,
                         int points_per_pixel, int32_t* idx, float* zbuf, float* dists, void* workspace,
                         size_t workspace_bytes, void* stream);

/*
 * Backward for L = <grad_zbuf, zbuf> + <grad_dists, dists> with the choice
 * of points held fixed: dL/dz_p sums grad_zbuf over p's slots and
 * dL/d(x_p, y_p) sums 2 grad_dists (x_p - px, y_p - py).  grad_points (P,3)
 * float32 is overwritten; grad_zbuf or grad_dists may be NULL (no term).
 * idx must be the output of rasterize_points_fwd for these points, cloud
 * ranges, size and radius: each point's slots are looked up among the pixels
 * its disc covers, so a slot naming a point at a pixel it does not cover is
 * ignored.  flags: 0 (sort the points again) or RAST_BWD_REUSE_FORWARD (take
 * the sorted points from the forward's workspace, unchanged since; a
 * workspace last used by another call is detected from its signature, the
 * gradient is then left zero and rast_query_status reports RAST_EREUSE).
 */
int rasterize_points_bwd(const float* points, int64_t P, const int64_t* cloud_to_first_idx,
                         const int64_t* num_points_per_cloud, int N, int H, int W, float radius,
                         int points_per_pixel, int flags, const int32_t* idx, const float* grad_zbuf,
                         const float* grad_dists, float* grad_points, void* workspace, size_t workspace_bytes,
                         void* stream);

/*
 * Point compositing (paper, Section 3.3) over npix pixels of K slots with
 * features (P,D) float32 (D in [1, RAST_COMPOSITE_DMAX]).  For a pixel whose
 * slots k hold points idx_k with opacities alpha_k, in slot order (nearest
 * first):
 *   RAST_COMPOSITE_ALPHA: image = sum_k alpha_k prod_{j<k} (1 - alpha_j) f_{idx_k}
 *   RAST_COMPOSITE_NORM:  image = sum_k alpha_k f_{idx_k} / sum_k alpha_k
 *                         (0 where the opacities sum to <= 0)
 * Slots with idx < 0 or idx >= P take no part.  weights (npix,K) float32
 * holds the opacities, or, with RAST_COMPOSITE_FROM_DISTS or-ed into mode,
 * the rasterizer's squared distances d, the opacity being
 * alpha = 1 - d / radius^2 (radius > 0).  image (npix,D) is overwritten.
 * features may be NULL: every feature of every point is then 1 (silhouette
 * compositing, the paper's boolean features), and no table is read; P still
 * bounds the valid ids.
 */
#define RAST_COMPOSITE_ALPHA 0
#define RAST_COMPOSITE_NORM 1
#define RAST_COMPOSITE_FROM_DISTS 2
#define RAST_COMPOSITE_DMAX 8
int points_composite_fwd(const int32_t* idx, const float* weights, const float* features, int64_t P, int64_t npix,
                         int K, int D, int mode, float radius, float* image, void* stream);

/*
 * Backward of points_composite_fwd for L = <grad_image, image>, with
 * g_k = <grad_image, f_{idx_k}> and T_k = prod_{j<k} (1 - alpha_j):
 *   ALPHA: dL/dalpha_k = T_k (g_k - R_k), R_k = sum_{i>k} alpha_i g_i prod_{k<j<i} (1 - alpha_j);
 *          dL/df_{idx_k} += alpha_k T_k grad_image
 *   NORM:  dL/dalpha_k = (g_k - <grad_image, image>) / S, S = sum_k alpha_k;
 *          dL/df_{idx_k} += alpha_k grad_image / S   (nothing where S <= 0)
 * grad_weights (npix,K) is overwritten with dL/dalpha_k, or dL/dd_k =
 * -dL/dalpha_k / radius^2 in RAST_COMPOSITE_FROM_DISTS mode; 0 for slots that
 * take no part.  grad_features (P,D) is overwritten, or NULL (not computed;
 * it must be NULL when features is); its sums are formed with float atomics,
 * so their rounding order varies.
 */
int points_composite_bwd(const int32_t* idx, const float* weights, const float* features, int64_t P, int64_t npix,
                         int K, int D, int mode, float radius, const float* grad_image, float* grad_weights,
                         float* grad_features, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RAST_H */
