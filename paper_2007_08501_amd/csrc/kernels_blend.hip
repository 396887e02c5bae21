// kernels_blend.hip -- silhouette blend (paper, Section 3.2, Algorithm 1) and
// its backward, one lane per pixel, for gfx950.
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
