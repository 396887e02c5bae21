// kernels_blend.hip -- silhouette blend (paper, Section 3.2, Algorithm 1),
// softmax blend (Algorithm 2) and their backwards, for gfx950: the
// silhouette blend spreads a pixel's slots over a group of lanes, the softmax
// blend takes one lane per pixel.
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

// A pixel's K slots are spread over L lanes of a wave, four consecutive slots
// per lane (L the power of two with 4 L >= K, 64 / L pixels per wave), so
// that consecutive lanes read consecutive words: each lane combines its own
// slots and only the per-lane products cross lanes (segmented scans of
// log2(L) steps).  One lane per pixel walking its K words would make every
// load instruction touch 64 different rows (a 200-byte stride at K = 50).
constexpr int kBlendQ = 4;  // consecutive slots per lane
// four words at 4-byte alignment (a pixel's slots start at any word)
typedef int bi32x4 __attribute__((ext_vector_type(4), aligned(4)));
typedef float bf32x4 __attribute__((ext_vector_type(4), aligned(4)));

// The lane's slots of pixel p: whether each holds a face, and d / sigma.
__device__ __forceinline__ void blend_slots(const int32_t* __restrict__ p2f, const float* __restrict__ d, int64_t p,
                                            int64_t P, int K, int sub, float inv_sigma, bool (&on)[kBlendQ],
                                            float (&x)[kBlendQ]) {
    const int64_t o = p * K + kBlendQ * sub;
    if (p < P && kBlendQ * (sub + 1) <= K) {
        const bi32x4 vi = *reinterpret_cast<const bi32x4*>(p2f + o);
        const bf32x4 vd = *reinterpret_cast<const bf32x4*>(d + o);
#pragma unroll
        for (int i = 0; i < kBlendQ; ++i) {
            on[i] = vi[i] >= 0;
            x[i] = vd[i] * inv_sigma;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kBlendQ; ++i) {
            const bool in = p < P && kBlendQ * sub + i < K;
            on[i] = in && p2f[o + i] >= 0;
            x[i] = in ? d[o + i] * inv_sigma : 0.0f;
        }
    }
}

template <int L>
__device__ __forceinline__ float blend_seg_prod(float v) {
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) v *= __shfl_xor(v, m, L);
    return v;
}

// product over the lower / the higher lanes of the segment (1 for none)
template <int L>
__device__ __forceinline__ float blend_excl_prefix(float t, int sub) {
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
        const float u = __shfl_up(t, m, L);
        if (sub >= m) t *= u;
    }
    const float e = __shfl_up(t, 1, L);
    return sub == 0 ? 1.0f : e;
}
template <int L>
__device__ __forceinline__ float blend_excl_suffix(float t, int sub) {
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
        const float u = __shfl_down(t, m, L);
        if (sub + m < L) t *= u;
    }
    const float e = __shfl_down(t, 1, L);
    return sub == L - 1 ? 1.0f : e;
}

template <int L>
__global__ __launch_bounds__(256) void blend_fwd_kernel(const int32_t* __restrict__ p2f, const float* __restrict__ d,
                                                        int64_t P, int K, float inv_sigma, float* __restrict__ alpha) {
    constexpr int PPW = 64 / L;
    const int lane = threadIdx.x & 63, sub = lane & (L - 1), grp = lane / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p0 = wave * PPW; p0 < P; p0 += nwaves * PPW) {
        const int64_t p = p0 + grp;
        bool on[kBlendQ];
        float x[kBlendQ];
        blend_slots(p2f, d, p, P, K, sub, inv_sigma, on, x);
        float t = 1.0f;  // product of 1 - prob_k over the lane's slots
#pragma unroll
        for (int i = 0; i < kBlendQ; ++i)
            if (on[i]) t *= sigmoidf(x[i]);
        t = blend_seg_prod<L>(t);
        if (sub == 0 && p < P) alpha[p] = 1.0f - t;
    }
}

// d alpha / d d_k = -(1/sigma) prob_k (1 - prob_k) prod_{j<k} (1 - prob_j)
// prod_{j>k} (1 - prob_j): the products of the other slots come from the
// lane's own prefix and suffix and the exclusive scans of the lane products
// (no division by 1 - prob_k, which underflows deep inside a face).
template <int L>
__global__ __launch_bounds__(256) void blend_bwd_kernel(const int32_t* __restrict__ p2f, const float* __restrict__ d,
                                                        const float* __restrict__ ga, int64_t P, int K, float inv_sigma,
                                                        float* __restrict__ gd) {
    constexpr int PPW = 64 / L;
    const int lane = threadIdx.x & 63, sub = lane & (L - 1), grp = lane / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p0 = wave * PPW; p0 < P; p0 += nwaves * PPW) {
        const int64_t p = p0 + grp;
        bool on[kBlendQ];
        float x[kBlendQ];
        blend_slots(p2f, d, p, P, K, sub, inv_sigma, on, x);
        float om[kBlendQ];  // 1 - prob_k (1 for an empty slot)
        float t = 1.0f;
#pragma unroll
        for (int i = 0; i < kBlendQ; ++i) {
            om[i] = on[i] ? sigmoidf(x[i]) : 1.0f;
            t *= om[i];
        }
        float pre = blend_excl_prefix<L>(t, sub);
        const float lsuf = blend_excl_suffix<L>(t, sub);
        const float g = p < P ? ga[p] : 0.0f;
        float out[kBlendQ];
#pragma unroll
        for (int i = 0; i < kBlendQ; ++i) {
            float suf = lsuf;
#pragma unroll
            for (int j = i + 1; j < kBlendQ; ++j) suf *= om[j];
            out[i] = on[i] ? -g * inv_sigma * sigmoidf(-x[i]) * om[i] * pre * suf : 0.0f;
            pre *= om[i];
        }
        const int64_t o = p * K + kBlendQ * sub;
        if (p < P && kBlendQ * (sub + 1) <= K) {
            *reinterpret_cast<bf32x4*>(gd + o) = bf32x4{out[0], out[1], out[2], out[3]};
        } else {
#pragma unroll
            for (int i = 0; i < kBlendQ; ++i)
                if (p < P && kBlendQ * sub + i < K) gd[o + i] = out[i];
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

// lanes per pixel: the power of two L with 4 L >= K (K <= 64)
static int blend_lanes(int K) {
    int L = 1;
    while (kBlendQ * L < K) L <<= 1;
    return L;
}

static unsigned blend_grid(int64_t P, int L) {
    const int64_t waves = (P + 64 / L - 1) / (64 / L);
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    return (unsigned)(blocks > 0 ? blocks : 1);
}

hipError_t launch_blend_fwd(const int32_t* p2f, const float* d, int64_t P, int K, float sigma, float* alpha,
                            hipStream_t s) {
    if (P == 0) return hipSuccess;
    const int L = blend_lanes(K);
    const dim3 grid(blend_grid(P, L));
#define RAST_BLEND_FWD(LL) \
    case LL: hipLaunchKernelGGL(blend_fwd_kernel<LL>, grid, dim3(256), 0, s, p2f, d, P, K, 1.0f / sigma, alpha); break;
    switch (L) {
        RAST_BLEND_FWD(1) RAST_BLEND_FWD(2) RAST_BLEND_FWD(4) RAST_BLEND_FWD(8) RAST_BLEND_FWD(16)
        default: return hipErrorInvalidValue;
    }
#undef RAST_BLEND_FWD
    return hipGetLastError();
}

hipError_t launch_blend_bwd(const int32_t* p2f, const float* d, const float* ga, int64_t P, int K, float sigma,
                            float* gd, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const int L = blend_lanes(K);
    const dim3 grid(blend_grid(P, L));
#define RAST_BLEND_BWD(LL)                                                                                       \
    case LL:                                                                                                     \
        hipLaunchKernelGGL(blend_bwd_kernel<LL>, grid, dim3(256), 0, s, p2f, d, ga, P, K, 1.0f / sigma, gd); \
        break;
    switch (L) {
        RAST_BLEND_BWD(1) RAST_BLEND_BWD(2) RAST_BLEND_BWD(4) RAST_BLEND_BWD(8) RAST_BLEND_BWD(16)
        default: return hipErrorInvalidValue;
    }
#undef RAST_BLEND_BWD
    return hipGetLastError();
}

}  // namespace rast
