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
// e^{-i pi k / 2N}); the inverse runs the same steps backwards.  The
// sequences are real, so a workgroup packs two rows into one complex
// transform and transforms it in LDS (self-sorting radix-8 passes, N <= 4096,
// powers of two); columns are rows of a transposed copy.  Per tile: DCT of the rows,
// transpose, DCT of the rows again (the spectrum, transposed); per scale:
// weighted inverse DCT of its rows, transpose, inverse DCT of the rows into
// stack plane k.  Arithmetic in FP32 with twiddles and weights built in
// FP64.
#include <math.h>
#include <stdint.h>

#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int FT = 512;  // threads per row workgroup (two rows)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS slot of complex sample i: one pad slot per 8, so that the strided
// writes of the first radix-8 passes (stride 8 and 64 samples) spread over
// the banks.
__device__ __forceinline__ int px(int i) { return i + (i >> 3); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * (-i) forward, a * (+i) inverse
template <bool INV>
__device__ __forceinline__ float2 rot_i(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Radix-R DFT of v in registers (R = 2, 4, 8); INV uses e^{+2 pi i / R}.
template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2 (&v)[R]);

template <>
__device__ __forceinline__ void dft_r<2, false>(float2 (&v)[2]) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <>
__device__ __forceinline__ void dft_r<2, true>(float2 (&v)[2]) { dft_r<2, false>(v); }

template <bool INV>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
    const float2 t3 = rot_i<INV>(csub(x1, x3));
    x0 = cadd(t0, t2);
    x1 = cadd(t1, t3);
    x2 = csub(t0, t2);
    x3 = csub(t1, t3);
}
template <>
__device__ __forceinline__ void dft_r<4, false>(float2 (&v)[4]) { dft4<false>(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void dft_r<4, true>(float2 (&v)[4]) { dft4<true>(v[0], v[1], v[2], v[3]); }

template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    constexpr float c = 0.70710678118654752f;
    // o_k times e^{-+ i pi k / 4}
    o1 = INV ? make_float2(c * (o1.x - o1.y), c * (o1.x + o1.y))
             : make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));
    o2 = rot_i<INV>(o2);
    o3 = INV ? make_float2(-c * (o3.x + o3.y), c * (o3.x - o3.y))
             : make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}
template <>
__device__ __forceinline__ void dft_r<8, false>(float2 (&v)[8]) { dft8<false>(v); }
template <>
__device__ __forceinline__ void dft_r<8, true>(float2 (&v)[8]) { dft8<true>(v); }

// One Stockham (self-sorting) pass of radix R over buf[0..n): sub-transforms
// of length Ns are merged into length Ns R.  Item j reads buf[j + r n / R],
// turns input r by e^{-+2 pi i (j mod Ns) r / (Ns R)} (1 in the first pass,
// Ns = 1), takes the radix-R DFT
// and writes buf[(j / Ns) Ns R + (j mod Ns) + r Ns].  Every item is read
// into registers before any is written (in place).  At most two items per
// thread: n / R <= FT for every pass of a transform up to 4096 points.
constexpr int PASS_ITEMS = 1;
static_assert(FFT_MAX_N <= 4096 && FFT_MAX_N / 8 <= PASS_ITEMS * FT,
              "a radix-8 pass of the longest transform fits the items per thread");

template <int R, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, int n, int Ns,
                                              const float2* __restrict__ tw, int nmax) {
    const int m = n / R;
    float2 v[PASS_ITEMS][R];
#pragma unroll
    for (int i = 0; i < PASS_ITEMS; ++i) {
        const int j = threadIdx.x + i * FT;
        if (j < m) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[px(j + r * m)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PASS_ITEMS; ++i) {
        const int j = threadIdx.x + i * FT;
        if (j < m) {
            const int jm = j & (Ns - 1);
            if (Ns > 1) {
                // e^{-2 pi i jm r / (Ns R)}: powers 1, 2, 4 from the table,
                // the others as products of two
                const int step = jm * (nmax / (Ns * R));
                float2 w[R];
                w[1] = tw[step];
                if constexpr (R >= 4) {
                    w[2] = tw[2 * step];
                    w[3] = cmul(w[1], w[2]);
                }
                if constexpr (R == 8) {
                    w[4] = tw[4 * step];
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    if (INV) w[r].y = -w[r].y;
                    v[i][r] = cmul(v[i][r], w[r]);
                }
            }
            dft_r<R, INV>(v[i]);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[px(base + r * Ns)] = v[i][r];
        }
    }
    __syncthreads();
}

// Complex FFT of buf[0..n) in LDS, natural order in and out (n a power of
// two up to 4096; no 1/n).  log2 n = 3 q + e: one radix-2^e pass, then q
// radix-8 passes.  tw[k] = e^{-2 pi i k / nmax}, k < nmax.  The caller
// synchronises after filling buf.
template <bool INV>
__device__ void fft_block(float2* buf, int n, int logn, const float2* __restrict__ tw, int nmax) {
    int Ns = 1;
    if (logn % 3 == 1) {
        stockham_pass<2, INV>(buf, n, Ns, tw, nmax);
        Ns = 2;
    } else if (logn % 3 == 2) {
        stockham_pass<4, INV>(buf, n, Ns, tw, nmax);
        Ns = 4;
    }
    for (int p = 0; p < logn / 3; ++p) {
        stockham_pass<8, INV>(buf, n, Ns, tw, nmax);
        Ns *= 8;
    }
}

// Position of sample i in the even/odd reordering: x[2m] -> v[m],
// x[2m+1] -> v[n-1-m].
__device__ __forceinline__ int dct_perm(int i, int n) { return (i & 1) ? n - 1 - (i >> 1) : (i >> 1); }

// Four consecutive samples of a row as floats (u8 codes as u / 255).
__device__ __forceinline__ float4 load4(const uint8_t* p) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(p);
    constexpr float s = 1.0f / 255.0f;
    return make_float4(static_cast<float>(u & 0xffu) * s, static_cast<float>((u >> 8) & 0xffu) * s,
                       static_cast<float>((u >> 16) & 0xffu) * s, static_cast<float>(u >> 24) * s);
}
__device__ __forceinline__ float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float load1(const uint8_t* p) { return static_cast<float>(*p) / 255.0f; }
__device__ __forceinline__ float load1(const float* p) { return *p; }

// Row accesses in groups of four (VEC: rows of a multiple of 4 samples with
// 16-byte aligned float, 4-byte aligned u8 starts): up to V4 groups per
// thread, all loads issued before the first LDS store.
constexpr int V4 = FFT_MAX_N / 4 / FT;

// DCT-II of rows of length n (power of two, n <= nmax), two rows per
// workgroup packed as the real and imaginary parts of one complex FFT: row
// r of the input at src + r pitch (u8 codes read as u/255, or floats), the
// coefficients to dst + r n.  With Z the FFT of the packed sequence,
// V_a[k] = (Z[k] + conj Z[n-k]) / 2 and V_b[k] = (Z[k] - conj Z[n-k]) / 2i,
// and C[k] = Re(V[k] e^{-i pi k / 2n}).  q[k] = e^{-i pi k / (2 nmax)}.
template <typename T, bool VEC>
__global__ __launch_bounds__(FT) void dct_rows_kernel(const T* __restrict__ src, long long pitch,
                                                      int rows, int n, int logn,
                                                      float* __restrict__ dst,
                                                      const float2* __restrict__ tw,
                                                      const float2* __restrict__ q, int nmax) {
    extern __shared__ float2 buf[];
    const int r0 = 2 * blockIdx.x;
    const bool two = r0 + 1 < rows;
    const T* ra = src + static_cast<long long>(r0) * pitch;
    const T* rb = ra + pitch;
    if constexpr (VEC) {
        // x[4t] -> v[2t], x[4t+1] -> v[n-1-2t], x[4t+2] -> v[2t+1], x[4t+3] -> v[n-2-2t]
        const int n4 = n >> 2;
        float4 xa[V4], xb[V4];
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int t = threadIdx.x + u * FT;
            if (t < n4) {
                xa[u] = load4(ra + 4 * t);
                xb[u] = two ? load4(rb + 4 * t) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int t = threadIdx.x + u * FT;
            if (t < n4) {
                buf[px(2 * t)] = make_float2(xa[u].x, xb[u].x);
                buf[px(n - 1 - 2 * t)] = make_float2(xa[u].y, xb[u].y);
                buf[px(2 * t + 1)] = make_float2(xa[u].z, xb[u].z);
                buf[px(n - 2 - 2 * t)] = make_float2(xa[u].w, xb[u].w);
            }
        }
    } else {
        for (int i = threadIdx.x; i < n; i += FT)
            buf[px(dct_perm(i, n))] = make_float2(load1(ra + i), two ? load1(rb + i) : 0.0f);
    }
    __syncthreads();
    fft_block<false>(buf, n, logn, tw, nmax);
    const int qs = nmax / n;
    float* oa = dst + static_cast<long long>(r0) * n;
    float* ob = oa + n;
    auto coef = [&](int k, float& ca, float& cb) {
        const float2 z = buf[px(k)], zr = buf[px((n - k) & (n - 1))];
        // V_a = (z + conj zr) / 2, V_b = -i (z - conj zr) / 2
        const float2 va = make_float2(0.5f * (z.x + zr.x), 0.5f * (z.y - zr.y));
        const float2 vb = make_float2(0.5f * (z.y + zr.y), -0.5f * (z.x - zr.x));
        const float2 w = q[k * qs];
        ca = va.x * w.x - va.y * w.y;
        cb = vb.x * w.x - vb.y * w.y;
    };
    if constexpr (VEC) {
        for (int t = threadIdx.x; t < (n >> 2); t += FT) {
            float4 a, b;
            coef(4 * t, a.x, b.x);
            coef(4 * t + 1, a.y, b.y);
            coef(4 * t + 2, a.z, b.z);
            coef(4 * t + 3, a.w, b.w);
            reinterpret_cast<float4*>(oa)[t] = a;
            if (two) reinterpret_cast<float4*>(ob)[t] = b;
        }
    } else {
        for (int k = threadIdx.x; k < n; k += FT) {
            float a, b;
            coef(k, a, b);
            oa[k] = a;
            if (two) ob[k] = b;
        }
    }
}

// Inverse of the DCT-II above for rows of length n, two rows per workgroup
// packed into one complex inverse FFT; coefficient u of row r is first
// multiplied by the scale's weight (Weights) when one is given.  Per row
// V[k] = e^{i pi k / 2n} (C[k] - i C[n-k]) with C[n] = 0; the packed
// spectrum V_a + i V_b transforms back to x_a + i x_b (times n).  The two
// (weighted) coefficient rows are staged in LDS as floats first, so that
// both C[k] and C[n-k] come from there.  Output row r to dst + r dst_pitch.
// Per-scale weights of the first inverse pass: row r, coefficient u get
// norm (g[r sx] h[u sy] + h[r sx] g[u sy]); g == nullptr: no weights.
struct Weights {
    const float* g = nullptr;
    const float* h = nullptr;
    int sx = 0, sy = 0;
    float norm = 0.0f;
};

template <bool VEC>
__global__ __launch_bounds__(FT) void idct_rows_kernel(const float* __restrict__ src, int rows,
                                                       int n, int logn, Weights W,
                                                       float* __restrict__ dst,
                                                       long long dst_pitch,
                                                       const float2* __restrict__ tw,
                                                       const float2* __restrict__ q, int nmax) {
    extern __shared__ float2 buf[];
    float* fa = reinterpret_cast<float*>(buf);  // row a coefficients, [0, n)
    float* fb = fa + n;                         // row b, [n, 2n)
    const int r0 = 2 * blockIdx.x;
    const bool two = r0 + 1 < rows;
    const float* ra = src + static_cast<long long>(r0) * n;
    const float* rb = ra + n;
    const bool weighted = W.g != nullptr;
    const float* __restrict__ b = W.h;  // coefficient u: a(r) b(u sy) + c(r) d(u sy)
    const float* __restrict__ d = W.g;
    const int sy = W.sy;
    const float a0 = weighted ? W.norm * W.g[r0 * W.sx] : 0.0f;
    const float c0 = weighted ? W.norm * W.h[r0 * W.sx] : 0.0f;
    const float a1 = weighted && two ? W.norm * W.g[(r0 + 1) * W.sx] : 0.0f;
    const float c1 = weighted && two ? W.norm * W.h[(r0 + 1) * W.sx] : 0.0f;
    if constexpr (VEC) {
        const int n4 = n >> 2;
        float4 xa[V4], xb[V4];
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int t = threadIdx.x + u * FT;
            if (t < n4) {
                xa[u] = reinterpret_cast<const float4*>(ra)[t];
                xb[u] = two ? reinterpret_cast<const float4*>(rb)[t]
                            : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int t = threadIdx.x + u * FT;
            if (t < n4) {
                float4 wa = make_float4(1.0f, 1.0f, 1.0f, 1.0f), wb = wa;
                if (weighted) {
                    const int k = 4 * t * sy;
                    const float b0 = b[k], b1 = b[k + sy], b2 = b[k + 2 * sy], b3 = b[k + 3 * sy];
                    const float d0 = d[k], d1 = d[k + sy], d2 = d[k + 2 * sy], d3 = d[k + 3 * sy];
                    wa = make_float4(a0 * b0 + c0 * d0, a0 * b1 + c0 * d1, a0 * b2 + c0 * d2,
                                     a0 * b3 + c0 * d3);
                    wb = make_float4(a1 * b0 + c1 * d0, a1 * b1 + c1 * d1, a1 * b2 + c1 * d2,
                                     a1 * b3 + c1 * d3);
                }
                reinterpret_cast<float4*>(fa)[t] =
                    make_float4(xa[u].x * wa.x, xa[u].y * wa.y, xa[u].z * wa.z, xa[u].w * wa.w);
                reinterpret_cast<float4*>(fb)[t] =
                    make_float4(xb[u].x * wb.x, xb[u].y * wb.y, xb[u].z * wb.z, xb[u].w * wb.w);
            }
        }
    } else {
        for (int k = threadIdx.x; k < n; k += FT) {
            const float va = ra[k], vb = two ? rb[k] : 0.0f;
            fa[k] = weighted ? va * (a0 * b[k * sy] + c0 * d[k * sy]) : va;
            fb[k] = weighted ? vb * (a1 * b[k * sy] + c1 * d[k * sy]) : vb;
        }
    }
    __syncthreads();
    // packed spectrum into registers, then over the staged rows
    const int qs = nmax / n;
    float2 z[4 * V4];
#pragma unroll
    for (int u = 0; u < 4 * V4; ++u) {
        const int k = threadIdx.x + u * FT;
        if (k < n) {
            const float2 w = q[k * qs];  // e^{-i pi k / 2n}; its conjugate is wanted
            const float ca = fa[k], cb = fb[k];
            const float cna = k ? fa[n - k] : 0.0f, cnb = k ? fb[n - k] : 0.0f;
            // conj(w) (C[k] - i C[n-k])
            const float2 va = make_float2(w.x * ca - w.y * cna, -w.x * cna - w.y * ca);
            const float2 vb = make_float2(w.x * cb - w.y * cnb, -w.x * cnb - w.y * cb);
            z[u] = make_float2(va.x - vb.y, va.y + vb.x);  // V_a + i V_b
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4 * V4; ++u) {
        const int k = threadIdx.x + u * FT;
        if (k < n) buf[px(k)] = z[u];
    }
    __syncthreads();
    fft_block<true>(buf, n, logn, tw, nmax);
    const float inv_n = 1.0f / static_cast<float>(n);
    float* oa = dst + static_cast<long long>(r0) * dst_pitch;
    float* ob = oa + dst_pitch;
    if constexpr (VEC) {
        for (int t = threadIdx.x; t < (n >> 2); t += FT) {
            const float2 z0 = buf[px(2 * t)], z1 = buf[px(n - 1 - 2 * t)];
            const float2 z2 = buf[px(2 * t + 1)], z3 = buf[px(n - 2 - 2 * t)];
            reinterpret_cast<float4*>(oa)[t] =
                make_float4(z0.x * inv_n, z1.x * inv_n, z2.x * inv_n, z3.x * inv_n);
            if (two)
                reinterpret_cast<float4*>(ob)[t] =
                    make_float4(z0.y * inv_n, z1.y * inv_n, z2.y * inv_n, z3.y * inv_n);
        }
    } else {
        for (int i = threadIdx.x; i < n; i += FT) {
            const float2 zz = buf[px(dct_perm(i, n))];
            oa[i] = zz.x * inv_n;
            if (two) ob[i] = zz.y * inv_n;
        }
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

// Spectral weights of every scale at the plan's longest transform nmax:
// lambda_t(u) = t_0 + 2 sum_{j=1}^{R} t_j cos(pi u j / nmax), u < nmax, for
// t in {g, h}, in double (angles reduced exactly: u j mod 2 nmax).  Layout
// [k][g, h][nmax].  A side n = nmax / 2^s takes every 2^s-th weight, since
// cos(pi u j / n) = cos(pi (2^s u) j / nmax).
__global__ void spectral_kernel(const double* __restrict__ taps, const int* __restrict__ tap_off,
                                const int* __restrict__ radii, int K, int nmax,
                                float* __restrict__ out) {
    const long long total = static_cast<long long>(K) * 2 * nmax;
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(i / (2 * nmax));
        const int rem = static_cast<int>(i - static_cast<long long>(k) * 2 * nmax);
        const int which = rem / nmax, u = rem - which * nmax;  // which: 0 g, 1 h
        const int R = radii[k];
        const double* t = taps + tap_off[k] + which * (R + 1);  // one-sided t_0 .. t_R
        double sum = t[0];
        const long long period = 2LL * nmax;
        for (int j = 1; j <= R; ++j) {
            const long long m = (static_cast<long long>(u) * j) % period;
            sum += 2.0 * t[j] * cospi(static_cast<double>(m) / nmax);
        }
        out[i] = static_cast<float>(sum);
    }
}

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

bool fft_size_ok(int n) { return n >= 1 && n <= FFT_MAX_N && (n & (n - 1)) == 0; }

size_t fft_workspace_floats(int h, int w) {
    // P / D / Q transform buffers
    return 3 * static_cast<size_t>(h) * w;
}

hipError_t build_fft_spectra(const double* taps, const int* tap_off, const int* radii, int K,
                             int nmax, float* lam, hipStream_t s) {
    spectral_kernel<<<1024, 256, 0, s>>>(taps, tap_off, radii, K, nmax, lam);
    return hipGetLastError();
}

hipError_t launch_fft_log_stack(const FftTables& T, int in_dtype, const void* img, int h, int w,
                                int64_t pitch, float* stack, float* ws, hipStream_t s) {
    const size_t hw = static_cast<size_t>(h) * w;
    float* P = ws;            // h x w
    float* D = ws + hw;       // w x h
    float* Q = ws + 2 * hw;   // w x h, then h x w
    const int lh = log2i(h), lw = log2i(w);
    const size_t lds_w = sizeof(float2) * (w + (w >> 3)), lds_h = sizeof(float2) * (h + (h >> 3));
    const dim3 tg_hw((w + 31) / 32, (h + 31) / 32), tg_wh((h + 31) / 32, (w + 31) / 32);
    const unsigned gh = (h + 1) / 2, gw = (w + 1) / 2;  // two rows per workgroup
    // groups of four: rows of >= 4 samples; the workspace and the per-scale
    // planes are 16-byte aligned then (h w a multiple of 4)
    auto aligned = [](const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; };
    const bool vw = w >= 4 && aligned(ws, 16), vh = h >= 4 && aligned(ws, 16);
    const size_t esz = in_dtype == MHFD_U8 ? 1 : 4;
    const bool vin = vw && pitch % 4 == 0 && aligned(img, 4 * esz);
    const bool vout = vw && aligned(stack, 16);
    if (in_dtype == MHFD_U8) {
        const uint8_t* src = static_cast<const uint8_t*>(img);
        if (vin)
            dct_rows_kernel<uint8_t, true><<<gh, FT, lds_w, s>>>(src, pitch, h, w, lw, P, T.tw, T.q, T.nmax);
        else
            dct_rows_kernel<uint8_t, false><<<gh, FT, lds_w, s>>>(src, pitch, h, w, lw, P, T.tw, T.q, T.nmax);
    } else {
        const float* src = static_cast<const float*>(img);
        if (vin)
            dct_rows_kernel<float, true><<<gh, FT, lds_w, s>>>(src, pitch, h, w, lw, P, T.tw, T.q, T.nmax);
        else
            dct_rows_kernel<float, false><<<gh, FT, lds_w, s>>>(src, pitch, h, w, lw, P, T.tw, T.q, T.nmax);
    }
    transpose_kernel<<<tg_hw, 256, 0, s>>>(P, h, w, Q);  // Q: w x h
    if (vh)  // D[v][u]: row v = x frequency, column u = y frequency
        dct_rows_kernel<float, true><<<gw, FT, lds_h, s>>>(Q, h, w, h, lh, D, T.tw, T.q, T.nmax);
    else
        dct_rows_kernel<float, false><<<gw, FT, lds_h, s>>>(Q, h, w, h, lh, D, T.tw, T.q, T.nmax);
    const int sx = T.nmax / w, sy = T.nmax / h;  // weight strides of the two sides
    for (int k = 0; k < T.K; ++k) {
        const float* gl = T.lam + static_cast<size_t>(k) * 2 * T.nmax;
        const float* hl = gl + T.nmax;
        float* plane = stack + static_cast<size_t>(k) * hw;
        // row v of D (x frequency), coefficient u (y frequency):
        // s sigma^2 (lambda_g(v) lambda_h(u) + lambda_h(v) lambda_g(u))
        const Weights wt{gl, hl, sx, sy, T.norm[k]};
        if (vh)
            idct_rows_kernel<true><<<gw, FT, lds_h, s>>>(D, w, h, lh, wt, Q, h, T.tw, T.q, T.nmax);
        else
            idct_rows_kernel<false><<<gw, FT, lds_h, s>>>(D, w, h, lh, wt, Q, h, T.tw, T.q, T.nmax);
        transpose_kernel<<<tg_wh, 256, 0, s>>>(Q, w, h, P);  // P: h x w
        if (vout)
            idct_rows_kernel<true><<<gh, FT, lds_w, s>>>(P, h, w, lw, Weights{}, plane, w, T.tw,
                                                         T.q, T.nmax);
        else
            idct_rows_kernel<false><<<gh, FT, lds_w, s>>>(P, h, w, lw, Weights{}, plane, w, T.tw,
                                                          T.q, T.nmax);
    }
    return hipGetLastError();
}

}  // namespace mhfd
