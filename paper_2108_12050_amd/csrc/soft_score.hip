// Soft focus score and its gradient: the kernels around the shared strip
// kernel.
//
//   S_b = 1/(K H W) sum_k sum_{y,x} softplus(beta (|r_k| - tau)),
//   r_k = sigma_k^2 Lap(G_sigma_k * I_b).
//
// Taps depend on the trainable sigmas, which live on the device, so they are
// synthesised here in double (no host round trip), each scale's kernel radius
// floor(truncate sigma + 0.5) taken from its current sigma, and launched at
// the padded radius of the plan's sigma cap (taps beyond the radius are
// zero).  Four tap sets per scale feed the strip
// kernel, whose operator is hcol (*)_y (grow (*)_x I) + gcol (*)_y (hrow (*)_x I):
//   FWD  (g, h, sigma^2 g, sigma^2 h)   r = sigma^2 Lap
//   D1   (g, h', g, h')                 the sigma-derivative of the Laplacian
//   D2   (g', h, g', h)                   is D1 + D2 (product rule on
//                                         h(y) g(x) + g(y) h(x))
//   ADJ  (g, h, g, h)                   the Laplacian operator itself, which is
//                                       its own adjoint under half-sample
//                                       reflection (each 1-D border-handled
//                                       convolution is a symmetric matrix)
// with primes the sigma-derivatives at fixed support:
//   g'_j = g_j (j^2 - V) / sigma^3,   V' = (M4 - V^2) / sigma^3,
//   h'_j = [(j^2 - V) g'_j - V' g_j] / sigma^4 - 4 (j^2 - V) g_j / sigma^5.
#include <math.h>

#include "mhfd_internal.h"

namespace mhfd {

namespace {

__global__ void soft_taps_kernel(const float* __restrict__ sigmas, SoftTapLayout lay,
                                 float* __restrict__ taps, int32_t* __restrict__ err) {
    const int k = threadIdx.x;
    const double s = k < lay.K ? static_cast<double>(sigmas[k]) : 1.0;
    const int P = k < lay.K ? lay.padded[k] : 1;
    // radius from the current sigma; accepted within (0, sigma_cap] and the
    // launch radius (comparisons are false for NaN)
    const double rr = floor(static_cast<double>(lay.truncate) * s + 0.5);
    const bool ok = k >= lay.K || (s > 0.0 && s <= static_cast<double>(lay.sigma_cap) && rr <= P);
    const int bad = __syncthreads_or(!ok);
    if (err && threadIdx.x == 0) *err = bad ? MHFD_FOCUS_BAD_SIGMA : 0;
    if (k >= lay.K) return;
    const int R = ok ? static_cast<int>(rr) : 0;
    float* base = taps + lay.offset[k];
    const int run = P + 1;  // floats per tap run
    const int blk = 4 * run;  // floats per tap set
    double z = 0.0, V = 0.0, M4 = 0.0;
    for (int j = 0; j <= R; ++j) {
        const double e = exp(-static_cast<double>(j) * j / (2.0 * s * s));
        z += j == 0 ? e : 2.0 * e;
    }
    for (int j = 1; j <= R; ++j) {
        const double gj = exp(-static_cast<double>(j) * j / (2.0 * s * s)) / z;
        const double j2 = static_cast<double>(j) * j;
        V += 2.0 * j2 * gj;
        M4 += 2.0 * j2 * j2 * gj;
    }
    const double s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s;
    const double Vd = (M4 - V * V) / s3;
    for (int j = 0; j <= P; ++j) {
        double g = 0.0, h = 0.0, gd = 0.0, hd = 0.0;
        if (j <= R) {
            const double j2 = static_cast<double>(j) * j;
            g = exp(-j2 / (2.0 * s2)) / z;
            const double q = j2 - V;
            h = q * g / s4;
            gd = g * q / s3;
            hd = (q * gd - Vd * g) / s4 - 4.0 * q * g / s5;
        }
        auto put = [&](int set, int r, double v) {
            base[set * blk + r * run + j] = ok ? static_cast<float>(v) : 0.0f;
        };
        // FWD
        put(0, 0, g);
        put(0, 1, h);
        put(0, 2, s2 * g);
        put(0, 3, s2 * h);
        // D1
        put(1, 0, g);
        put(1, 1, hd);
        put(1, 2, g);
        put(1, 3, hd);
        // D2
        put(2, 0, gd);
        put(2, 1, h);
        put(2, 2, gd);
        put(2, 3, h);
        // ADJ
        put(3, 0, g);
        put(3, 1, h);
        put(3, 2, g);
        put(3, 3, h);
    }
}

// S_b = sum of the softplus partials of image b / (K H W), in a fixed order.
// Partials are laid out per class launch c as [image][block] from base[c].
__global__ void soft_finish_kernel(const double* __restrict__ partial, SoftPartials sp, int batch,
                                   double inv_khw, float* __restrict__ scores) {
    const int b = blockIdx.x;
    if (b >= batch) return;
    __shared__ double sh[256];
    double t = 0.0;
    for (int c = 0; c < sp.n; ++c) {
        const double* q = partial + sp.base[c] + static_cast<long long>(b) * sp.blocks[c];
        for (int i = threadIdx.x; i < sp.blocks[c]; i += blockDim.x) t += q[i];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int d = blockDim.x / 2; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) scores[b] = static_cast<float>(sh[0] * inv_khw);
}

// Per pixel of scale k: w = gbar_b/(KHW) beta sigmoid(beta(|r| - tau)) sgn(r);
// sigma partial += w (2 r / sigma + sigma^2 d); r is overwritten by the
// cotangent c = w sigma^2.  One double partial per workgroup.
constexpr int COT_T = 256;

__global__ __launch_bounds__(COT_T) void soft_cotangent_kernel(
    float* __restrict__ r, const float* __restrict__ d, long long n_per_image, int batch,
    const float* __restrict__ sigmas, int k, const float* __restrict__ gbar, double inv_khw,
    float beta, float tau, double* __restrict__ partial) {
    __shared__ double sh[COT_T / 64];
    const double sg = static_cast<double>(sigmas[k]);
    const float sgf = sigmas[k];
    const float s2 = sgf * sgf;
    const long long n = n_per_image * batch;
    double acc = 0.0;
    for (long long i = blockIdx.x * static_cast<long long>(COT_T) + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * COT_T) {
        const int b = static_cast<int>(i / n_per_image);
        const float rv = r[i];
        const float z = beta * (fabsf(rv) - tau);
        const float sig = 1.0f / (1.0f + expf(-z));
        const float sgn = rv > 0.0f ? 1.0f : (rv < 0.0f ? -1.0f : 0.0f);
        const float w = static_cast<float>(gbar[b] * inv_khw) * beta * sig * sgn;
        acc += static_cast<double>(w) * (2.0 * static_cast<double>(rv) / sg +
                                         static_cast<double>(s2) * static_cast<double>(d[i]));
        r[i] = w * s2;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < COT_T / 64; ++w) t += sh[w];
        partial[blockIdx.x] = t;
    }
}

__global__ void sigma_grad_finish_kernel(const double* __restrict__ partial, int nb, int K,
                                         float* __restrict__ dsig) {
    const int k = blockIdx.x;
    if (k >= K) return;
    __shared__ double sh[256];
    double t = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) t += partial[static_cast<long long>(k) * nb + i];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int d = blockDim.x / 2; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) dsig[k] = static_cast<float>(sh[0]);
}

}  // namespace

int soft_cotangent_blocks() { return 2048; }

hipError_t launch_soft_taps(const float* sigmas, const SoftTapLayout& lay, float* taps,
                            int32_t* err, hipStream_t s) {
    static_assert(MHFD_MAX_SCALES <= 64, "one thread per scale");
    soft_taps_kernel<<<1, 64, 0, s>>>(sigmas, lay, taps, err);
    return hipGetLastError();
}

hipError_t launch_soft_finish(const double* partial, const SoftPartials& sp, int batch,
                              double inv_khw, float* scores, hipStream_t s) {
    soft_finish_kernel<<<batch, 256, 0, s>>>(partial, sp, batch, inv_khw, scores);
    return hipGetLastError();
}

hipError_t launch_soft_cotangent(float* r, const float* d, long long n_per_image, int batch,
                                 const float* sigmas, int k, const float* gbar, double inv_khw,
                                 float beta, float tau, double* partial, hipStream_t s) {
    soft_cotangent_kernel<<<soft_cotangent_blocks(), COT_T, 0, s>>>(
        r, d, n_per_image, batch, sigmas, k, gbar, inv_khw, beta, tau, partial);
    return hipGetLastError();
}

hipError_t launch_sigma_grad_finish(const double* partial, int nb, int K, float* dsig,
                                    hipStream_t s) {
    sigma_grad_finish_kernel<<<K, 256, 0, s>>>(partial, nb, K, dsig);
    return hipGetLastError();
}

}  // namespace mhfd
