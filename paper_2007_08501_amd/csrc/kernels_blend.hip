// kernels_blend.hip -- silhouette blend (paper, Section 3.2, Algorithm 1),
// softmax blend (Algorithm 2) and their backwards, one lane per pixel, for
// gfx950.
//
// Silhouette:
//   prob_k = sigmoid(-d_k / sigma) where the slot holds a face, else 0
//   alpha  = 1 - prod_k (1 - prob_k)
//   d alpha / d d_k = -(1/sigma) prob_k (1 - prob_k) prod_{j != k} (1 - prob_j)
// 1 - prob_k is evaluated as sigmoid(+d_k / sigma) so that it keeps its
// relative accuracy where prob_k is close to 1 (deep inside a face).
#include "device.hpp"
#include "launch.hpp"

namespace rast {

__device__ __forceinline__ float sigmoidf(float x) {
    // 1 / (1 + exp(-x)), evaluated on the side where exp does not overflow
    if (x >= 0.0f) return 1.0f / (1.0f + expf(-x));
    float e = expf(x);
    return e / (1.0f + e);
}

__global__ __launch_bounds__(256) void blend_fwd_kernel(const int32_t* __restrict__ p2f, const float* __restrict__ d,
                                                        int64_t P, int K, float inv_sigma, float* __restrict__ alpha) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float prod = 1.0f;
    for (int k = 0; k < K; ++k) {
        int64_t o = p * K + k;
        if (p2f[o] >= 0) prod *= sigmoidf(d[o] * inv_sigma);
    }
    alpha[p] = 1.0f - prod;
}

// Two sweeps over the pixel's K slots: the first stores the suffix products
// prod_{j > k} (1 - prob_j) into grad_dists, the second walks forward with the
// prefix product and overwrites each entry with the gradient.
__global__ __launch_bounds__(256) void blend_bwd_kernel(const int32_t* __restrict__ p2f, const float* __restrict__ d,
                                                        const float* __restrict__ ga, int64_t P, int K, float inv_sigma,
                                                        float* __restrict__ gd) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float suf = 1.0f;
    for (int k = K - 1; k >= 0; --k) {
        int64_t o = p * K + k;
        gd[o] = suf;
        if (p2f[o] >= 0) suf *= sigmoidf(d[o] * inv_sigma);
    }
    float g = ga[p];
    float pre = 1.0f;
    for (int k = 0; k < K; ++k) {
        int64_t o = p * K + k;
        if (p2f[o] >= 0) {
            float x = d[o] * inv_sigma;
            float prob = sigmoidf(-x);
            float om = sigmoidf(x);
            gd[o] = -g * inv_sigma * prob * om * pre * gd[o];
            pre *= om;
        } else {
            gd[o] = 0.0f;
        }
    }
}

// Softmax blend: prob_k = sigmoid(-d_k / sigma), zinv_k = (zfar - z_k) / (zfar - znear),
// w_k = prob_k exp((zinv_k - max_j zinv_j) / gamma), image = sum_k w_k c_k / sum_k w_k.
// Empty slots take no part; a pixel whose weights sum to 0 is 0.  CB is a
// compile-time bound on the channel count C.
// The exponent is evaluated as (min_j z_j - z_k) / ((zfar - znear) gamma),
// which equals (zinv_k - max zinv) / gamma: forming zinv first would round
// zfar - z (about zfar) and then divide that rounding by a small gamma.
struct SoftmaxArgs {
    const int32_t* p2f;
    const float* z;
    const float* d;
    const float* col;
    int64_t P;
    int K, C;
    float inv_sigma;
    float zscale;  // 1 / ((zfar - znear) gamma)
};

// Smallest depth over the pixel's filled slots (the largest zinv); 0 when there are none.
__device__ __forceinline__ float softmax_zmin(const SoftmaxArgs& a, int64_t p) {
    float m = INFINITY;
    for (int k = 0; k < a.K; ++k) {
        const int64_t o = p * a.K + k;
        if (a.p2f[o] >= 0) m = fminf(m, a.z[o]);
    }
    return m == INFINITY ? 0.0f : m;
}

__device__ __forceinline__ float softmax_weight(const SoftmaxArgs& a, int64_t o, float zmin) {
    return sigmoidf(-a.d[o] * a.inv_sigma) * expf((zmin - a.z[o]) * a.zscale);
}

// Weight sum and the blended colour of pixel p.
template <int CB>
__device__ __forceinline__ float softmax_pixel(const SoftmaxArgs& a, int64_t p, float m, float (&out)[CB]) {
    float W = 0.0f;
#pragma unroll
    for (int c = 0; c < CB; ++c) out[c] = 0.0f;
    for (int k = 0; k < a.K; ++k) {
        const int64_t o = p * a.K + k;
        if (a.p2f[o] < 0) continue;
        const float w = softmax_weight(a, o, m);
        W += w;
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c < a.C) out[c] = fmaf(w, a.col[o * a.C + c], out[c]);
    }
    const float inv = W > 0.0f ? 1.0f / W : 0.0f;
#pragma unroll
    for (int c = 0; c < CB; ++c) out[c] *= inv;
    return W;
}

template <int CB>
__global__ __launch_bounds__(256) void softmax_fwd_kernel(SoftmaxArgs a, float* __restrict__ img) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    float out[CB];
    softmax_pixel<CB>(a, p, softmax_zmin(a, p), out);
#pragma unroll
    for (int c = 0; c < CB; ++c)
        if (c < a.C) img[p * a.C + c] = out[c];
}

// With G_k = sum_c g_c (c_kc - image_c) / W:
//   dL/dd_k = -G_k w_k (1 - prob_k) / sigma, dL/dz_k = -G_k w_k / (gamma (zfar - znear)),
//   dL/dc_kc = g_c w_k / W.  The max-zinv shift cancels in the normalised weights.
template <int CB>
__global__ __launch_bounds__(256) void softmax_bwd_kernel(SoftmaxArgs a, const float* __restrict__ gimg,
                                                          float* __restrict__ gz, float* __restrict__ gd,
                                                          float* __restrict__ gc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const float m = softmax_zmin(a, p);
    float out[CB];
    const float W = softmax_pixel<CB>(a, p, m, out);
    const float inv = W > 0.0f ? 1.0f / W : 0.0f;
    float g[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) g[c] = c < a.C ? gimg[p * a.C + c] : 0.0f;
    for (int k = 0; k < a.K; ++k) {
        const int64_t o = p * a.K + k;
        float w = 0.0f, G = 0.0f, om = 0.0f;
        if (a.p2f[o] >= 0 && W > 0.0f) {
            w = softmax_weight(a, o, m);
            om = sigmoidf(a.d[o] * a.inv_sigma);
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < a.C) G = fmaf(g[c], a.col[o * a.C + c] - out[c], G);
            G *= inv;
        }
        if (gd) gd[o] = -G * w * om * a.inv_sigma;
        if (gz) gz[o] = -G * w * a.zscale;
        if (gc) {
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < a.C) gc[o * a.C + c] = g[c] * w * inv;
        }
    }
}

static SoftmaxArgs softmax_args(const int32_t* p2f, const float* z, const float* d, const float* col, int64_t P,
                                int K, int C, float sigma, float gamma, float znear, float zfar) {
    SoftmaxArgs a;
    a.p2f = p2f;
    a.z = z;
    a.d = d;
    a.col = col;
    a.P = P;
    a.K = K;
    a.C = C;
    a.inv_sigma = 1.0f / sigma;
    a.zscale = (float)(1.0 / (((double)zfar - (double)znear) * (double)gamma));
    return a;
}

hipError_t launch_softmax_fwd(const int32_t* p2f, const float* z, const float* d, const float* col, int64_t P, int K,
                              int C, float sigma, float gamma, float znear, float zfar, float* img, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const SoftmaxArgs a = softmax_args(p2f, z, d, col, P, K, C, sigma, gamma, znear, zfar);
    const dim3 grid((unsigned)((P + 255) / 256));
    if (C <= 4)
        hipLaunchKernelGGL(softmax_fwd_kernel<4>, grid, dim3(256), 0, s, a, img);
    else
        hipLaunchKernelGGL(softmax_fwd_kernel<8>, grid, dim3(256), 0, s, a, img);
    return hipGetLastError();
}

hipError_t launch_softmax_bwd(const int32_t* p2f, const float* z, const float* d, const float* col, int64_t P, int K,
                              int C, float sigma, float gamma, float znear, float zfar, const float* gimg, float* gz,
                              float* gd, float* gc, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const SoftmaxArgs a = softmax_args(p2f, z, d, col, P, K, C, sigma, gamma, znear, zfar);
    const dim3 grid((unsigned)((P + 255) / 256));
    if (C <= 4)
        hipLaunchKernelGGL(softmax_bwd_kernel<4>, grid, dim3(256), 0, s, a, gimg, gz, gd, gc);
    else
        hipLaunchKernelGGL(softmax_bwd_kernel<8>, grid, dim3(256), 0, s, a, gimg, gz, gd, gc);
    return hipGetLastError();
}

hipError_t launch_blend_fwd(const int32_t* p2f, const float* d, int64_t P, int K, float sigma, float* alpha,
                            hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(blend_fwd_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, p2f, d, P, K,
                       1.0f / sigma, alpha);
    return hipGetLastError();
}

hipError_t launch_blend_bwd(const int32_t* p2f, const float* d, const float* ga, int64_t P, int K, float sigma,
                            float* gd, hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(blend_bwd_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, p2f, d, ga, P, K,
                       1.0f / sigma, gd);
    return hipGetLastError();
}

}  // namespace rast
