// Scale-normalised LoG of one scale, streamed down vertical strips.
//
// R = s sigma^2 (h (*)_y A + g (*)_y B),  A = g (*)_x I,  B = h (*)_x I
// (the 2-D Gaussian of section 2.2 factorises as g(x) g(y), so its Laplacian
// is h(x) g(y) + g(x) h(y)).  Every scale is independent of the others
// (section 3 makes the same observation for the per-scale filtering), so
// scales are separate launches.
//
// One workgroup owns a strip of TW output columns and a segment of rows.  It
// walks down the segment in chunks of CH rows:
//   stage   CH input rows, columns [x0 - R, x0 + TW + R), into LDS, applying
//           the half-sample reflection at the image borders;
//   row     pass: A and B of those rows (TW columns) into an LDS ring that
//           holds the last CH + 2R rows, so every row pass is done once per
//           segment and not once per output tile;
//   column  pass: CH output rows from the ring, with the Laplacian sum and the
//           s sigma^2 factor folded into the column taps; written to HBM.
// The row pass keeps 8 + 2R input values of one row in registers and forms
// 8 outputs from symmetric pair sums (one add feeds both the g and the h
// product).  The column pass slides down the ring, one LDS read of (A, B)
// per row feeding 8 output rows.  Taps are wave-uniform and live in scalar
// registers.
#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int TW = 64;   // output columns per strip (one per lane in the column pass)
constexpr int CH = 32;   // rows per chunk
constexpr int NT = 256;  // threads per workgroup (4 waves)
constexpr int PX = 8;    // row-pass outputs per thread
constexpr int QY = 8;    // column-pass outputs per thread

template <typename T>
__device__ __forceinline__ float load_px(const T* p);
template <>
__device__ __forceinline__ float load_px<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float load_px<uint8_t>(const uint8_t* p) {
    return static_cast<float>(*p) / 255.0f;
}

template <int R, typename T>
__global__ __launch_bounds__(NT) void log_strip_kernel(const T* __restrict__ img, int H, int W,
                                                       long long pitch,
                                                       const float* __restrict__ taps,
                                                       float* __restrict__ out,
                                                       long long out_pitch, int seg_rows) {
    constexpr int NB = TW + 2 * R;  // staged input columns
    constexpr int S = CH + 2 * R;   // ring rows
    static_assert(R % 4 == 0, "padded radius");
    __shared__ __attribute__((aligned(16))) float in_s[CH * NB];
    __shared__ __attribute__((aligned(16))) float2 ab_s[S * TW];

    const float* __restrict__ g_row = taps;
    const float* __restrict__ h_row = taps + (R + 1);
    const float* __restrict__ g_col = taps + 2 * (R + 1);
    const float* __restrict__ h_col = taps + 3 * (R + 1);

    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TW;
    const int ys = blockIdx.y * seg_rows;
    const int ye = min(ys + seg_rows, H);
    const bool interior_x = (x0 - R >= 0) && (x0 + TW + R <= W);

    // Input rows [r0, r0 + n), columns [x0 - R, x0 + TW + R).
    auto stage = [&](int r0, int n) {
        for (int idx = tid; idx < n * NB; idx += NT) {
            const int row = idx / NB;
            const int c = idx - row * NB;
            const int gy = reflect_index(r0 + row, H);
            const int gx = interior_x ? x0 - R + c : reflect_index(x0 - R + c, W);
            in_s[row * NB + c] = load_px(img + static_cast<long long>(gy) * pitch + gx);
        }
    };

    // A, B of rows [r0, r0 + n) into the ring.  Ring slot of image row r is
    // (r - ys + R) mod S.
    auto rowpass = [&](int r0, int n) {
        const int row = tid >> 3;
        const int cg = tid & 7;
        if (row < n) {
            float v[PX + 2 * R];
            const float4* src = reinterpret_cast<const float4*>(in_s + row * NB + cg * PX);
#pragma unroll
            for (int m = 0; m < (PX + 2 * R) / 4; ++m) {
                const float4 t = src[m];
                v[4 * m + 0] = t.x;
                v[4 * m + 1] = t.y;
                v[4 * m + 2] = t.z;
                v[4 * m + 3] = t.w;
            }
            float a[PX], b[PX];
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                a[p] = g_row[0] * v[p + R];
                b[p] = h_row[0] * v[p + R];
            }
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const float gj = g_row[j];
                const float hj = h_row[j];
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    const float sum = v[p + R - j] + v[p + R + j];
                    a[p] = fmaf(gj, sum, a[p]);
                    b[p] = fmaf(hj, sum, b[p]);
                }
            }
            const int slot = (r0 + row - ys + R) % S;
            float2* dst = ab_s + slot * TW + cg * PX;
#pragma unroll
            for (int p = 0; p < PX; ++p) dst[p] = make_float2(a[p], b[p]);
        }
    };

    // Output rows [yc, yc + CH): wave w owns rows yc + 8w .. yc + 8w + 7, lane = column.
    auto colpass = [&](int yc) {
        const int lane = tid & 63;
        const int q0 = __builtin_amdgcn_readfirstlane(tid >> 6) * QY;
        float acc[QY];
#pragma unroll
        for (int q = 0; q < QY; ++q) acc[q] = 0.0f;
        // slot of image row yc + q0 - R
        const int base = (yc + q0 - ys) % S;
#pragma unroll
        for (int t = 0; t < QY + 2 * R; ++t) {
            int slot = base + t;
            slot = slot >= S ? slot - S : slot;
            const float2 ab = ab_s[slot * TW + lane];
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int i = q + R - t;  // row offset of this input for output q
                if (i >= -R && i <= R) {
                    const int ai = i < 0 ? -i : i;
                    acc[q] = fmaf(h_col[ai], ab.x, acc[q]);
                    acc[q] = fmaf(g_col[ai], ab.y, acc[q]);
                }
            }
        }
        const int x = x0 + lane;
        if (x < W) {
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int y = yc + q0 + q;
                if (y < ye) out[static_cast<long long>(y) * out_pitch + x] = acc[q];
            }
        }
    };

    // Prologue: rows [ys - R, ys + R).
    for (int r0 = ys - R; r0 < ys + R; r0 += CH) {
        const int n = min(CH, ys + R - r0);
        stage(r0, n);
        __syncthreads();
        rowpass(r0, n);
        __syncthreads();
    }
    for (int yc = ys; yc < ye; yc += CH) {
        stage(yc + R, CH);
        __syncthreads();  // also: every wave has finished the previous column pass
        rowpass(yc + R, CH);
        __syncthreads();
        colpass(yc);
    }
}

template <int R>
hipError_t launch_r(int in_dtype, const void* img, int h, int w, int64_t pitch, const float* taps,
                    float* out, int64_t out_pitch, int seg_rows, hipStream_t s) {
    dim3 grid((w + TW - 1) / TW, (h + seg_rows - 1) / seg_rows);
    if (in_dtype == MHFD_U8)
        log_strip_kernel<R, uint8_t><<<grid, NT, 0, s>>>(static_cast<const uint8_t*>(img), h, w,
                                                         pitch, taps, out, out_pitch, seg_rows);
    else
        log_strip_kernel<R, float><<<grid, NT, 0, s>>>(static_cast<const float*>(img), h, w,
                                                       pitch, taps, out, out_pitch, seg_rows);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_log_scale(int padded, int in_dtype, const void* img, int h, int w,
                            int64_t pitch, const float* taps, float* out, int64_t out_pitch,
                            int seg_rows, hipStream_t s) {
    switch (padded) {
#define MHFD_CASE(R) \
    case R:          \
        return launch_r<R>(in_dtype, img, h, w, pitch, taps, out, out_pitch, seg_rows, s);
        MHFD_CASE(4)
        MHFD_CASE(8)
        MHFD_CASE(12)
        MHFD_CASE(16)
        MHFD_CASE(20)
        MHFD_CASE(24)
        MHFD_CASE(28)
        MHFD_CASE(32)
        MHFD_CASE(36)
        MHFD_CASE(40)
        MHFD_CASE(44)
        MHFD_CASE(48)
        MHFD_CASE(52)
        MHFD_CASE(56)
        MHFD_CASE(60)
        MHFD_CASE(64)
#undef MHFD_CASE
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mhfd
