// kernels_bwd.hip -- backward of the rasterizer for gfx950.
//
// For every slot with a face, the barycentrics, z and the nearest edge are
// recomputed from the vertices (only the face ids are kept from the forward),
// the fragment gradients are chained to the nine coordinates of the face's
// vertices, and the result is added into grad_verts with float atomics.
//
// Derivatives (pixel p fixed, R_j = v_j - p, cross(u,v) = u.x v.y - u.y v.x):
//   e0 = cross(R1,R2), e1 = cross(R2,R0), e2 = cross(R0,R1), E = e0+e1+e2,
//   w_i = e_i / E.  With G_i = gbary_i + gzbuf * z_i and Gw = sum_i G_i w_i,
//   dL/dv_j(xy) = sum_i (G_i - Gw)/E * de_i/dv_j   (uses dE/dv = sum_i de_i/dv)
//   dL/dz_j     = gzbuf * w_j
//   dists = s d2 (s = -1 inside, +1 outside); on the nearest edge (s0, t) with
//   nearest point Q = R_s0 + u (R_t - R_s0) (relative to p):
//   d d2/d s0 = 2 (1-u) Q,  d d2/d t = 2 u Q.
#include "device.hpp"
#include "launch.hpp"

namespace rast {

struct BwdArgs {
    const float* verts;
    const int32_t* faces;
    const int32_t* p2f;
    const float* gz;
    const float* gb;
    const float* gd;
    float* grad;
    int64_t S;
    int64_t V, F;
    int H, W, K;
};

__global__ __launch_bounds__(256) void raster_bwd_kernel(BwdArgs a) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.S) return;
    int f = a.p2f[s];
    if (f < 0 || f >= a.F) return;  // an id outside [0, F) cannot come from the forward; ignore it
    int64_t pix = s / a.K;
    int64_t hw = (int64_t)a.H * a.W;
    int rem = (int)(pix % hw);
    int r = rem / a.W, c = rem - r * a.W;
    const Pix p = make_pix(r, c, a.H, a.W);
    int vi[3] = {a.faces[3 * (int64_t)f], a.faces[3 * (int64_t)f + 1], a.faces[3 * (int64_t)f + 2]};
    if (vi[0] < 0 || vi[0] >= a.V || vi[1] < 0 || vi[1] >= a.V || vi[2] < 0 || vi[2] >= a.V) return;
    float P[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int x = 0; x < 3; ++x) P[j][x] = a.verts[3 * (int64_t)vi[j] + x];
    }
    FaceRec R = make_rec(P[0][0], P[0][1], P[0][2], P[1][0], P[1][1], P[1][2], P[2][0], P[2][1], P[2][2], 0.0f, 0);
    if (!R.ok()) return;
    Eval ev;
    eval_full(R, p, ev);
    float gzs = a.gz ? a.gz[s] : 0.0f;
    float gb0 = 0.0f, gb1 = 0.0f, gb2 = 0.0f;
    if (a.gb) {
        gb0 = a.gb[3 * s + 0];
        gb1 = a.gb[3 * s + 1];
        gb2 = a.gb[3 * s + 2];
    }
    float gds = a.gd ? a.gd[s] : 0.0f;
    float w[3] = {ev.w0, ev.w1, ev.w2};
    float G0 = gb0 + gzs * P[0][2];
    float G1 = gb1 + gzs * P[1][2];
    float G2 = gb2 + gzs * P[2][2];
    float Gw = G0 * w[0] + G1 * w[1] + G2 * w[2];
    float invE = R.invE();
    float H0 = (G0 - Gw) * invE, H1 = (G1 - Gw) * invE, H2 = (G2 - Gw) * invE;
    // vertex positions relative to the pixel, from the record's exact pieces
    float Rx[3], Ry[3];
    Rx[0] = -ev.sx;
    Ry[0] = -ev.sy;
    Rx[1] = Rx[0] + R.q1.x;
    Ry[1] = Ry[0] + R.q1.y;
    Rx[2] = Rx[0] + R.q1.z;
    Ry[2] = Ry[0] + R.q1.w;
    // de0/dR1 = (R2.y, -R2.x), de0/dR2 = (-R1.y, R1.x)
    // de1/dR2 = (R0.y, -R0.x), de1/dR0 = (-R2.y, R2.x)
    // de2/dR0 = (R1.y, -R1.x), de2/dR1 = (-R0.y, R0.x)
    float gx[3], gy[3];
    gx[0] = H1 * (-Ry[2]) + H2 * Ry[1];
    gy[0] = H1 * Rx[2] + H2 * (-Rx[1]);
    gx[1] = H0 * Ry[2] + H2 * (-Ry[0]);
    gy[1] = H0 * (-Rx[2]) + H2 * Rx[0];
    gx[2] = H0 * (-Ry[1]) + H1 * Ry[0];
    gy[2] = H0 * Rx[1] + H1 * (-Rx[0]);
    if (gds != 0.0f) {
        int e = ev.edge;
        int js = e, jt = e == 2 ? 0 : e + 1;
        float u = ev.u;
        float Qx = Rx[js] + u * (Rx[jt] - Rx[js]);
        float Qy = Ry[js] + u * (Ry[jt] - Ry[js]);
        float sg = ev.inside ? -gds : gds;
        float cs = 2.0f * (1.0f - u) * sg, ct = 2.0f * u * sg;
        // only the two endpoints of the nearest edge move d2
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float k = (j == js) ? cs : ((j == jt) ? ct : 0.0f);
            gx[j] += k * Qx;
            gy[j] += k * Qy;
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float* g = a.grad + 3 * (int64_t)vi[j];
        atomicAdd(g + 0, gx[j]);
        atomicAdd(g + 1, gy[j]);
        atomicAdd(g + 2, gzs * w[j]);
    }
}

hipError_t launch_backward(const float* verts, int64_t V, const int32_t* faces, int64_t F, int N, int H, int W, int K,
                           const int32_t* p2f, const float* gz, const float* gb, const float* gd, float* grad,
                           hipStream_t s, hipEvent_t eb, hipEvent_t ee) {
    hipError_t e = launch_fill_f32(grad, V * 3, 0.0f, s);
    if (e != hipSuccess) return e;
    BwdArgs a;
    a.verts = verts;
    a.faces = faces;
    a.p2f = p2f;
    a.gz = gz;
    a.gb = gb;
    a.gd = gd;
    a.grad = grad;
    a.S = (int64_t)N * H * W * K;
    a.V = V;
    a.F = F;
    a.H = H;
    a.W = W;
    a.K = K;
    if (a.S == 0) return hipSuccess;
    if (eb) hipEventRecord(eb, s);
    hipLaunchKernelGGL(raster_bwd_kernel, dim3((unsigned)((a.S + 255) / 256)), dim3(256), 0, s, a);
    if (ee) hipEventRecord(ee, s);
    return hipGetLastError();
}

}  // namespace rast
