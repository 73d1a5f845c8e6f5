// Soft focus score and its gradient: the kernels around the matrix-core
// (or, for launch radii above its limit, the strip) operator.
//
//   S_b = 1/(K H W) sum_k sum_{y,x} softplus(beta (|r_k| - tau)),
//   r_k = sigma_k^2 Lap(G_sigma_k * I_b).
//
// Taps depend on the trainable sigmas, which live on the device, so they are
// synthesised here in double (no host round trip), each scale's kernel radius
// floor(truncate sigma + 0.5) taken from its current sigma, and launched at
// the padded radius of the plan's sigma cap (taps beyond the radius are
// zero).  Four tap sets per scale, each (grow, hrow, gcol, hcol) for the
// operator hcol (*)_y (grow (*)_x I) + gcol (*)_y (hrow (*)_x I):
//   FWD  (g, h, sigma^2 g, sigma^2 h)   r = sigma^2 Lap
//   D1   (g, h, g', h')                 the sigma-derivative of the Laplacian
//   D2   (g', h', g, h)                   is D1 + D2 (product rule on
//                                         h(y) g(x) + g(y) h(x): D1 holds
//                                         h'(y) g(x) + g'(y) h(x), D2
//                                         h(y) g'(x) + g(y) h'(x)); D1 has
//                                         the row taps of FWD
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

// One workgroup per scale k (64 threads over the taps j = 0 .. P); workgroup
// 0 also writes the error word from every scale's acceptance.
__device__ __forceinline__ bool sigma_ok(double s, double truncate, double cap, int P) {
    // radius from the current sigma; accepted within (0, cap] and the launch
    // radius (comparisons are false for NaN)
    const double rr = floor(truncate * s + 0.5);
    return s > 0.0 && s <= cap && rr <= P;
}

// sum over the 64 lanes of the wave (the workgroup is one wave)
__device__ __forceinline__ double sum64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64) void soft_taps_kernel(const float* __restrict__ sigmas,
                                                       SoftTapLayout lay, float* __restrict__ taps,
                                                       int32_t* __restrict__ err) {
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const double trunc = static_cast<double>(lay.truncate);
    const double cap = static_cast<double>(lay.sigma_cap);
    if (k == 0 && err) {
        bool bad = false;
        for (int q = tid; q < lay.K; q += 64)
            bad |= !sigma_ok(static_cast<double>(sigmas[q]), trunc, cap, lay.padded[q]);
        bad = __any(bad);
        if (tid == 0) *err = bad ? MHFD_FOCUS_BAD_SIGMA : 0;
    }
    const double s = static_cast<double>(sigmas[k]);
    const int P = lay.padded[k];
    const bool ok = sigma_ok(s, trunc, cap, P);
    const int R = ok ? static_cast<int>(floor(trunc * s + 0.5)) : 0;
    float* base = taps + lay.offset[k];
    const int run = P + 1;  // floats per tap run
    const int blk = 4 * run;  // floats per tap set
    double z = 0.0, V = 0.0, M4 = 0.0;
    for (int j = tid; j <= R; j += 64) {
        const double e = exp(-static_cast<double>(j) * j / (2.0 * s * s));
        z += j == 0 ? e : 2.0 * e;
    }
    z = sum64(z);
    for (int j = tid; j <= R; j += 64) {
        if (j == 0) continue;
        const double gj = exp(-static_cast<double>(j) * j / (2.0 * s * s)) / z;
        const double j2 = static_cast<double>(j) * j;
        V += 2.0 * j2 * gj;
        M4 += 2.0 * j2 * j2 * gj;
    }
    V = sum64(V);
    M4 = sum64(M4);
    const double s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s;
    const double Vd = (M4 - V * V) / s3;
    for (int j = tid; j <= P; j += 64) {
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
        put(1, 1, h);
        put(1, 2, gd);
        put(1, 3, hd);
        // D2
        put(2, 0, gd);
        put(2, 1, hd);
        put(2, 2, g);
        put(2, 3, h);
        // ADJ
        put(3, 0, g);
        put(3, 1, h);
        put(3, 2, g);
        put(3, 3, h);
    }
}

// Largest integer S with m 2^S <= limit (m > 0).
__device__ int pow2_fit_dev(double m, double limit) {
    int S = static_cast<int>(floor(log2(limit / m)));
    while (ldexp(m, S + 1) <= limit) ++S;
    while (ldexp(m, S) > limit) --S;
    return S;
}

__device__ __forceinline__ uint16_t half_of(float v) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(v));
}

// Matrix-core fragments of one (scale, tap set) per workgroup (blockIdx.x =
// scale, blockIdx.y = set) from the float tap runs grow, hrow, gcol, hcol of
// the strip layout, whose operator is hcol (*)_y (grow (*)_x I) +
// gcol (*)_y (hrow (*)_x I): row taps (grow, hrow), column taps (hcol for
// the grow intermediate, gcol for the hrow one).  The power-of-two factors
// follow the plan tables: fp32 input below 2^14, row intermediates at or
// below 2^15, the largest column tap at or below 2^14; each tap as an FP16
// pair hi + lo.  Fragment layout as the kernel reads it: row K-block kb,
// part t (0/1: grow hi/lo, 2/3: hrow hi/lo), lane (column n = lane & 15,
// group lane >> 4), 8 halves; then the column K-blocks likewise.
__global__ __launch_bounds__(256) void soft_frags_kernel(const float* __restrict__ taps,
                                                         SoftTapLayout lay, SoftFragLayout fl,
                                                         uint16_t* __restrict__ frags,
                                                         float* __restrict__ scales) {
    const int k = blockIdx.x, set = blockIdx.y;  // blockIdx.z: slice of the table
    const int P = lay.padded[k];
    const float* base = taps + lay.offset[k] + set * 4 * (P + 1);
    const float* grow = base;
    const float* hrow = base + (P + 1);
    const float* gcol = base + 2 * (P + 1);
    const float* hcol = base + 3 * (P + 1);
    __shared__ int sS[3];
    if (threadIdx.x == 0) {
        constexpr double in_max = 16384.0;
        double sg = 0.0, sh = 0.0;
        for (int j = 0; j <= P; ++j) {
            sg += (j ? 2.0 : 1.0) * fabs(static_cast<double>(grow[j]));
            sh += (j ? 2.0 : 1.0) * fabs(static_cast<double>(hrow[j]));
        }
        const int Sg = sg > 0.0 ? pow2_fit_dev(in_max * sg, 32768.0) : 0;
        const int Sh = sh > 0.0 ? pow2_fit_dev(in_max * sh, 32768.0) : 0;
        double cmax = 0.0;
        for (int j = 0; j <= P; ++j)
            cmax = fmax(cmax, fmax(fabs(ldexp(static_cast<double>(hcol[j]), -Sg)),
                                   fabs(ldexp(static_cast<double>(gcol[j]), -Sh))));
        const int Sc = cmax > 0.0 ? pow2_fit_dev(cmax, 16384.0) : 0;
        sS[0] = Sg;
        sS[1] = Sh;
        sS[2] = Sc;
        if (blockIdx.z == 0) scales[4 * k + set] = ldexpf(1.0f, -Sc);
    }
    __syncthreads();
    const int Sg = sS[0], Sh = sS[1], Sc = sS[2];
    const int nkr = fl.nkr[k], nkc = fl.nkc[k], rw8 = fl.rw8[k], rwc = fl.rwc[k];
    uint16_t* dst = frags + fl.off[k] + static_cast<long long>(set) * fl.halves[k];
    const int nrow = nkr * 4 * 64 * 8, ntot = (nkr + nkc) * 4 * 64 * 8;
    for (int e = blockIdx.z * blockDim.x + threadIdx.x; e < ntot; e += gridDim.z * blockDim.x) {
        const bool col = e >= nrow;
        const int f = col ? e - nrow : e;
        const int i = f & 7, lane = (f >> 3) & 63, t = (f >> 9) & 3, kb = f >> 11;
        const int n = lane & 15, gq = lane >> 4;
        int j;
        if (!col)
            j = 32 * kb + 8 * gq + i - rw8 - n;
        else
            j = 32 * kb + (i < 4 ? 4 * gq + i : 16 + 4 * gq + (i - 4)) - rwc - n;
        const int a = j < 0 ? -j : j;
        float v = 0.0f;
        if (a <= P) {
            if (!col)
                v = t < 2 ? ldexpf(grow[a], Sg) : ldexpf(hrow[a], Sh);
            else
                v = t < 2 ? ldexpf(ldexpf(hcol[a], -Sg), Sc) : ldexpf(ldexpf(gcol[a], -Sh), Sc);
        }
        const uint16_t hi = half_of(v);
        dst[e] = (t & 1) ? half_of(v - static_cast<float>(__builtin_bit_cast(_Float16, hi))) : hi;
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

// Workgroup row blockIdx.y is image b; the gridDim.x workgroups of the row
// stride over its pixels.  Partials laid out [image][workgroup]; with
// `cmax`, max |c| of image b as float bits (zero on entry) for the input
// scale of the adjoint on the matrix cores.
__global__ __launch_bounds__(COT_T) void soft_cotangent_kernel(
    float* __restrict__ r, const float* __restrict__ d, long long n_per_image,
    const float* __restrict__ sigmas, int k, const float* __restrict__ gbar, double inv_khw,
    float beta, float tau, double* __restrict__ partial, uint32_t* __restrict__ cmax) {
    __shared__ double sh[COT_T / 64];
    __shared__ float shm[COT_T / 64];
    const int b = blockIdx.y;
    const double sg = static_cast<double>(sigmas[k]);
    const float sgf = sigmas[k];
    const float s2 = sgf * sgf;
    const float wb = static_cast<float>(gbar[b] * inv_khw) * beta;
    float* rb = r + static_cast<long long>(b) * n_per_image;
    const float* db = d + static_cast<long long>(b) * n_per_image;
    double acc = 0.0;
    float m = 0.0f;
    for (long long i = blockIdx.x * static_cast<long long>(COT_T) + threadIdx.x; i < n_per_image;
         i += static_cast<long long>(gridDim.x) * COT_T) {
        const float rv = rb[i];
        const float z = beta * (fabsf(rv) - tau);
        const float sig = 1.0f / (1.0f + __expf(-z));
        const float sgn = rv > 0.0f ? 1.0f : (rv < 0.0f ? -1.0f : 0.0f);
        const float w = wb * sig * sgn;
        acc += static_cast<double>(w) * (2.0 * static_cast<double>(rv) / sg +
                                         static_cast<double>(s2) * static_cast<double>(db[i]));
        const float c = w * s2;
        rb[i] = c;
        m = fmaxf(m, fabsf(c));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        acc += __shfl_down(acc, o, 64);
        m = fmaxf(m, __shfl_down(m, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = acc;
        shm[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        float mm = 0.0f;
#pragma unroll
        for (int w = 0; w < COT_T / 64; ++w) {
            t += sh[w];
            mm = fmaxf(mm, shm[w]);
        }
        partial[static_cast<long long>(b) * gridDim.x + blockIdx.x] = t;
        if (cmax && mm > 0.0f) atomicMax(cmax + b, __float_as_uint(mm));
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

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void zero_f64_kernel(double* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

// Workgroups per image of the cotangent pass (about 2048 in all).
int cotangent_blocks_per_image(int batch) { return batch >= 2048 ? 1 : 2048 / batch; }

int soft_cotangent_blocks(int batch) { return cotangent_blocks_per_image(batch) * batch; }

hipError_t launch_soft_taps(const float* sigmas, const SoftTapLayout& lay, float* taps,
                            int32_t* err, hipStream_t s) {
    soft_taps_kernel<<<lay.K, 64, 0, s>>>(sigmas, lay, taps, err);
    return hipGetLastError();
}

hipError_t launch_soft_frags(const float* taps, const SoftTapLayout& lay, const SoftFragLayout& fl,
                             uint16_t* frags, float* scales, hipStream_t s) {
    soft_frags_kernel<<<dim3(fl.K, SOFT_SETS, 8), 256, 0, s>>>(taps, lay, fl, frags, scales);
    return hipGetLastError();
}

hipError_t launch_soft_finish(const double* partial, const SoftPartials& sp, int batch,
                              double inv_khw, float* scores, hipStream_t s) {
    soft_finish_kernel<<<batch, 256, 0, s>>>(partial, sp, batch, inv_khw, scores);
    return hipGetLastError();
}

hipError_t launch_soft_cotangent(float* r, const float* d, long long n_per_image, int batch,
                                 const float* sigmas, int k, const float* gbar, double inv_khw,
                                 float beta, float tau, double* partial, uint32_t* cmax,
                                 hipStream_t s) {
    if (cmax) zero_u32_kernel<<<(batch + 255) / 256, 256, 0, s>>>(cmax, batch);
    soft_cotangent_kernel<<<dim3(cotangent_blocks_per_image(batch), batch), COT_T, 0, s>>>(
        r, d, n_per_image, sigmas, k, gbar, inv_khw, beta, tau, partial, cmax);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    zero_f64_kernel<<<static_cast<unsigned>(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_sigma_grad_finish(const double* partial, int nb, int K, float* dsig,
                                    hipStream_t s) {
    sigma_grad_finish_kernel<<<K, 256, 0, s>>>(partial, nb, K, dsig);
    return hipGetLastError();
}

}  // namespace mhfd
