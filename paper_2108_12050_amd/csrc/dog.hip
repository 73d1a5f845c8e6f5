// The paper's own criterion (equation "dog" of section 2.2; equation
// "argmax" and Algorithm 1 of section 3) on Gaussian planes L_k (K x h x w,
// from the matrix-core kernel with Gaussian taps):
//
//   dog     per pixel DoG_i = t_i (L_{i+1} - L_i), i < K - 1, their maximum M
//           and its first argmax (the inner argmax over scale).  Reads the K
//           planes once and writes M (fp32) and the argmax (u8): HBM-bound,
//           4 K + 5 bytes per pixel;
//   (tail)  the detection tail run on M as a one-plane stack: with K = 1 the
//           3x3x3 window test is the 3x3 maxpool equality of the outer
//           argmaxlocal, with the plan's threshold, compaction and count;
//   label   the records' k and sigma from the argmax plane.
#include "mhfd_internal.h"

namespace mhfd {

namespace {

// Four adjacent pixels per thread (float4 loads of every plane) when the
// plane size is a multiple of 4 (planes then start 16-byte aligned), else one.
template <int V>
__global__ void dog_kernel(const float* __restrict__ L, int K, const float* __restrict__ sig,
                           long long n_px, float* __restrict__ M, uint8_t* __restrict__ arg) {
    typedef float Vec __attribute__((ext_vector_type(V)));
    const long long n_v = n_px / V;
    for (long long q = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; q < n_v;
         q += static_cast<long long>(gridDim.x) * blockDim.x) {
        Vec lo = reinterpret_cast<const Vec*>(L)[q];
        Vec best = static_cast<Vec>(-INFINITY);
        int bi[V];
#pragma unroll
        for (int c = 0; c < V; ++c) bi[c] = 0;
        for (int i = 0; i + 1 < K; ++i) {
            const Vec hi = reinterpret_cast<const Vec*>(L + (i + 1) * n_px)[q];
            const Vec d = sig[i] * (hi - lo);
#pragma unroll
            for (int c = 0; c < V; ++c)
                if (d[c] > best[c]) {
                    best[c] = d[c];
                    bi[c] = i;
                }
            lo = hi;
        }
        reinterpret_cast<Vec*>(M)[q] = best;
#pragma unroll
        for (int c = 0; c < V; ++c) arg[q * V + c] = static_cast<uint8_t>(bi[c]);
    }
}

__global__ void dog_label_kernel(mhfd_blob* __restrict__ blobs, int capacity,
                                 const mhfd_result* __restrict__ result,
                                 const uint8_t* __restrict__ arg, int w,
                                 const float* __restrict__ sig) {
    const long long n = min(result->n_blobs, static_cast<long long>(capacity));
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        mhfd_blob b = blobs[i];
        b.k = arg[static_cast<long long>(b.y) * w + b.x];
        b.sigma = sig[b.k];
        blobs[i] = b;
    }
}

}  // namespace

hipError_t launch_dog(const float* L, int K, const float* sigmas_dev, int h, int w, float* M,
                      uint8_t* arg, hipStream_t s) {
    const long long n = static_cast<long long>(h) * w;
    const bool v4 = n % 4 == 0 && reinterpret_cast<uintptr_t>(L) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(M) % 16 == 0;
    const long long blocks = ((v4 ? n / 4 : n) + 255) / 256;
    const int grid = blocks < 8192 ? static_cast<int>(blocks) : 8192;
    if (v4)
        dog_kernel<4><<<grid, 256, 0, s>>>(L, K, sigmas_dev, n, M, arg);
    else
        dog_kernel<1><<<grid, 256, 0, s>>>(L, K, sigmas_dev, n, M, arg);
    return hipGetLastError();
}

hipError_t launch_dog_label(mhfd_blob* blobs, int capacity, const mhfd_result* result,
                            const uint8_t* arg, int w, const float* sigmas_dev, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    dog_label_kernel<<<256, 256, 0, s>>>(blobs, capacity, result, arg, w, sigmas_dev);
    return hipGetLastError();
}

}  // namespace mhfd
