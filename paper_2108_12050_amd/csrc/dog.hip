// The paper's own criterion (section 4, equations "dog" and "argmax";
// Algorithm 1) on Gaussian planes L_k (K x h x w, from the matrix-core
// kernel with Gaussian taps):
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

__global__ void dog_kernel(const float* __restrict__ L, int K, const float* __restrict__ sig,
                           long long n_px, float* __restrict__ M, uint8_t* __restrict__ arg) {
    for (long long p = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; p < n_px;
         p += static_cast<long long>(gridDim.x) * blockDim.x) {
        float lo = L[p];
        float best = -INFINITY;
        int bi = 0;
        for (int i = 0; i + 1 < K; ++i) {
            const float hi = L[(i + 1) * n_px + p];
            const float d = sig[i] * (hi - lo);
            if (d > best) {
                best = d;
                bi = i;
            }
            lo = hi;
        }
        M[p] = best;
        arg[p] = static_cast<uint8_t>(bi);
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
    const long long blocks = (n + 255) / 256;
    dog_kernel<<<blocks < 8192 ? static_cast<int>(blocks) : 8192, 256, 0, s>>>(L, K, sigmas_dev,
                                                                                n, M, arg);
    return hipGetLastError();
}

hipError_t launch_dog_label(mhfd_blob* blobs, int capacity, const mhfd_result* result,
                            const uint8_t* arg, int w, const float* sigmas_dev, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    dog_label_kernel<<<256, 256, 0, s>>>(blobs, capacity, result, arg, w, sigmas_dev);
    return hipGetLastError();
}

}  // namespace mhfd
