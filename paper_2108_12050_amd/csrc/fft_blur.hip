// Scale-space operator in the frequency domain (plan mode MHFD_BLUR_FFT):
// the convolution of section 3 computed as a product of transforms, whose
// cost does not depend on the kernel radius.
//
// With half-sample symmetric borders the image is one period of a 2H x 2W
// even extension, so its discrete Fourier transform reduces to the 2-D
// DCT-II (no 4x extended array), and convolution with a symmetric kernel t
// (radius R, wrapped with period 2N, any R) multiplies DCT coefficient u by
//   lambda_t(u) = sum_{|j| <= R} t_j cos(pi u j / N).
// The LoG response of scale k, s sigma^2 (h(y) g(x) + g(y) h(x)) applied to
// I, is therefore
//   R_k = IDCT2( DCT2(I) * s sigma^2 (lambda_h(u) lambda_g(v) + lambda_g(u) lambda_h(v)) ).
//
// Each 1-D DCT-II of length N is one complex FFT of length N after the
// even/odd reordering v[n] = x[2n], v[N-1-n] = x[2n+1]: C[k] = Re(V[k]
// e^{-i pi k / 2N}); the inverse runs the same steps backwards.  A
// workgroup transforms one row in LDS (radix-2, N <= 4096, powers of two);
// columns are rows of a transposed copy.  Per tile: DCT of the rows,
// transpose, DCT of the rows again (the spectrum, transposed); per scale:
// weighted inverse DCT of its rows, transpose, inverse DCT of the rows into
// stack plane k.  Arithmetic in FP32 with twiddles and weights built in
// FP64.
#include <math.h>
#include <stdint.h>

#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int FT = 256;  // threads per row workgroup

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bit_reverse(int i, int logn) {
    return logn ? static_cast<int>(__brev(static_cast<unsigned>(i)) >> (32 - logn)) : 0;
}

// In-place radix-2 FFT of buf[0..N) (bit-reversed order on entry, natural
// order on exit).  tw[k] = e^{-2 pi i k / nmax}, k < nmax / 2; `inverse`
// conjugates the twiddles (no 1/N).
__device__ void fft_lds(float2* buf, int n, int logn, const float2* __restrict__ tw, int nmax,
                        bool inverse) {
    for (int s = 1; s <= logn; ++s) {
        __syncthreads();
        const int half = 1 << (s - 1);
        const int stride = nmax >> s;  // twiddle of index j in a span 2 half
        for (int b = threadIdx.x; b < (n >> 1); b += FT) {
            const int j = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + j;
            const int i1 = i0 + half;
            float2 w = tw[j * stride];
            if (inverse) w.y = -w.y;
            const float2 t = cmul(w, buf[i1]);
            const float2 u = buf[i0];
            buf[i0] = make_float2(u.x + t.x, u.y + t.y);
            buf[i1] = make_float2(u.x - t.x, u.y - t.y);
        }
    }
    __syncthreads();
}

// DCT-II of `rows` rows of length n (power of two, n <= nmax): row r of the
// input at src + r pitch (u8 codes read as u/255, or floats), the
// coefficients to dst + r n.  q[k] = e^{-i pi k / (2 nmax)}, k < nmax.
template <typename T>
__global__ __launch_bounds__(FT) void dct_rows_kernel(const T* __restrict__ src, long long pitch,
                                                      int n, int logn, float* __restrict__ dst,
                                                      const float2* __restrict__ tw,
                                                      const float2* __restrict__ q, int nmax) {
    extern __shared__ float2 buf[];
    const T* row = src + static_cast<long long>(blockIdx.x) * pitch;
    for (int i = threadIdx.x; i < n; i += FT) {
        float x;
        if constexpr (sizeof(T) == 1)
            x = static_cast<float>(row[i]) / 255.0f;
        else
            x = row[i];
        // x[2m] -> v[m], x[2m+1] -> v[n-1-m]
        const int m = (i & 1) ? n - 1 - (i >> 1) : (i >> 1);
        buf[bit_reverse(m, logn)] = make_float2(x, 0.0f);
    }
    fft_lds(buf, n, logn, tw, nmax, false);
    const int qs = nmax / n;
    float* out = dst + static_cast<long long>(blockIdx.x) * n;
    for (int k = threadIdx.x; k < n; k += FT) {
        const float2 v = buf[k];
        const float2 w = q[k * qs];
        out[k] = v.x * w.x - v.y * w.y;  // Re(V[k] e^{-i pi k / 2n})
    }
}

// Inverse DCT (of the DCT-II above) of rows of length n, each coefficient u
// of row r first multiplied by a(r) b(u) + c(r) d(u) when `a` is given:
// x = IDCT(C) to dst + r dst_pitch.
__global__ __launch_bounds__(FT) void idct_rows_kernel(const float* __restrict__ src, int n,
                                                       int logn, const float* __restrict__ a,
                                                       const float* __restrict__ b,
                                                       const float* __restrict__ c,
                                                       const float* __restrict__ d,
                                                       float* __restrict__ dst,
                                                       long long dst_pitch,
                                                       const float2* __restrict__ tw,
                                                       const float2* __restrict__ q, int nmax) {
    extern __shared__ float2 buf[];
    const int r = blockIdx.x;
    const float* row = src + static_cast<long long>(r) * n;
    const float ar = a ? a[r] : 0.0f, cr = a ? c[r] : 0.0f;
    auto coef = [&](int k) -> float {
        if (k >= n) return 0.0f;  // C[n] = 0
        const float v = row[k];
        return a ? v * (ar * b[k] + cr * d[k]) : v;
    };
    const int qs = nmax / n;
    for (int k = threadIdx.x; k < n; k += FT) {
        // V[k] = e^{i pi k / 2n} (C[k] - i C[n-k])
        const float ck = coef(k), cn = k ? coef(n - k) : 0.0f;
        const float2 w = q[k * qs];  // e^{-i pi k / 2n}; its conjugate is wanted
        const float2 z = make_float2(ck, -cn);
        buf[bit_reverse(k, logn)] = make_float2(w.x * z.x + w.y * z.y, w.x * z.y - w.y * z.x);
    }
    fft_lds(buf, n, logn, tw, nmax, true);
    const float inv_n = 1.0f / static_cast<float>(n);
    float* out = dst + static_cast<long long>(r) * dst_pitch;
    for (int i = threadIdx.x; i < n; i += FT) {
        const int m = (i & 1) ? n - 1 - (i >> 1) : (i >> 1);
        out[i] = buf[m].x * inv_n;
    }
}

// dst (cols x rows) = transpose of src (rows x cols), 32 x 32 tiles.
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ src, int rows,
                                                        int cols, float* __restrict__ dst) {
    __shared__ float t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int j = ty; j < 32; j += 8) {
        const int y = by + j, x = bx + tx;
        if (y < rows && x < cols) t[j][tx] = src[static_cast<long long>(y) * cols + x];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int x = bx + j, y = by + tx;  // dst row x, column y
        if (x < cols && y < rows) dst[static_cast<long long>(x) * rows + y] = t[tx][j];
    }
}

// Spectral weights of every scale for an h x w tile: for scale k and axis
// length n, lambda_t(u) = t_0 + 2 sum_{j=1}^{R} t_j cos(pi u j / n) for t in
// {g, h}, in double (angles reduced exactly: u j mod 2n).  Layout per scale
// (offset k * 2 (h + w)): g_y[h], h_y[h], g_x[w], h_x[w]; the x-axis arrays
// carry the normalisation s sigma^2.
__global__ void spectral_kernel(const double* __restrict__ taps, const int* __restrict__ tap_off,
                                const int* __restrict__ radii, const double* __restrict__ norm,
                                int K, int h, int w, float* __restrict__ out) {
    const int per = 2 * (h + w);
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
         i < static_cast<long long>(K) * per; i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(i / per);
        int u = static_cast<int>(i - static_cast<long long>(k) * per);
        int n, which;  // which: 0 g, 1 h
        bool xaxis;
        if (u < 2 * h) {
            n = h;
            which = u / h;
            u -= which * h;
            xaxis = false;
        } else {
            u -= 2 * h;
            n = w;
            which = u / w;
            u -= which * w;
            xaxis = true;
        }
        const int R = radii[k];
        const double* t = taps + tap_off[k] + which * (R + 1);  // one-sided t_0 .. t_R
        double s = t[0];
        const long long period = 2LL * n;
        for (int j = 1; j <= R; ++j) {
            const long long m = (static_cast<long long>(u) * j) % period;
            s += 2.0 * t[j] * cospi(static_cast<double>(m) / n);
        }
        if (xaxis) s *= norm[k];
        out[i] = static_cast<float>(s);
    }
}

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

bool fft_size_ok(int n) { return n >= 1 && n <= FFT_MAX_N && (n & (n - 1)) == 0; }

size_t fft_workspace_floats(int K, int h, int w) {
    // P / D / Q transform buffers (three h w) and the spectral weights
    return 3 * static_cast<size_t>(h) * w + static_cast<size_t>(K) * 2 * (h + w);
}

hipError_t launch_fft_log_stack(const FftTables& T, int in_dtype, const void* img, int h, int w,
                                int64_t pitch, float* stack, float* ws, hipStream_t s) {
    const size_t hw = static_cast<size_t>(h) * w;
    float* P = ws;            // h x w
    float* D = ws + hw;       // w x h
    float* Q = ws + 2 * hw;   // w x h, then h x w
    float* lam = ws + 3 * hw;
    const int lh = log2i(h), lw = log2i(w);
    const size_t lds_w = sizeof(float2) * w, lds_h = sizeof(float2) * h;
    const dim3 tg_hw((w + 31) / 32, (h + 31) / 32), tg_wh((h + 31) / 32, (w + 31) / 32);
    spectral_kernel<<<256, 256, 0, s>>>(T.taps, T.tap_off, T.radii, T.norm, T.K, h, w, lam);
    if (in_dtype == MHFD_U8)
        dct_rows_kernel<uint8_t><<<h, FT, lds_w, s>>>(static_cast<const uint8_t*>(img), pitch, w,
                                                      lw, P, T.tw, T.q, T.nmax);
    else
        dct_rows_kernel<float><<<h, FT, lds_w, s>>>(static_cast<const float*>(img), pitch, w, lw,
                                                    P, T.tw, T.q, T.nmax);
    transpose_kernel<<<tg_hw, 256, 0, s>>>(P, h, w, Q);                 // Q: w x h
    dct_rows_kernel<float><<<w, FT, lds_h, s>>>(Q, h, h, lh, D, T.tw, T.q, T.nmax);  // D[v][u]
    const int per = 2 * (h + w);
    for (int k = 0; k < T.K; ++k) {
        const float* L = lam + static_cast<size_t>(k) * per;
        const float* gy = L;
        const float* hy = L + h;
        const float* gx = L + 2 * h;
        const float* hx = L + 2 * h + w;
        // row v of D, coefficient u: gx(v) hy(u) + hx(v) gy(u)  (normalised)
        idct_rows_kernel<<<w, FT, lds_h, s>>>(D, h, lh, gx, hy, hx, gy, Q, h, T.tw, T.q, T.nmax);
        transpose_kernel<<<tg_wh, 256, 0, s>>>(Q, w, h, P);            // P: h x w
        idct_rows_kernel<<<h, FT, lds_w, s>>>(P, w, lw, nullptr, nullptr, nullptr, nullptr,
                                              stack + static_cast<size_t>(k) * hw, w, T.tw, T.q,
                                              T.nmax);
    }
    return hipGetLastError();
}

}  // namespace mhfd
