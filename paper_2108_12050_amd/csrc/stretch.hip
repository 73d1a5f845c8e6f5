// Histogram stretch of 8-bit images (section 3; Algorithm 1, first step):
// 0.175% of the pixels are saturated at each end and the codes between the
// two levels are mapped linearly onto [0, 1].
//
//   hist    256-bin histogram.  Every workgroup counts its rows into 32
//           copies of the histogram in LDS (lane l adds to copy l mod 32, bin
//           b's copies in 32 consecutive words, so equal codes in a wave
//           conflict at most 2 ways), then adds the sum of its copies to one
//           of n_copies global histograms (workgroup g to copy g mod
//           n_copies).  The global adds of all workgroups meet on 256 words
//           and are served one after another per word: with one global copy
//           they take more time than the counting itself, with 8 copies (one
//           per XCD under the round-robin dispatch of workgroups) little;
//   levels  one workgroup: sums the global copies (and writes the 256-bin
//           histogram where asked), then bin b's cumulative counts from
//           below and from above against q = 0.00175 N, compared in integers
//           (100000 count >= 175 N).  Below-counts are monotone in b, so the
//           low level is the number of bins whose count from below is still
//           short of q; the high level mirrors it from above.
//
// The mapping itself, clip((v - low) / (high - low), 0, 1), is applied where
// the codes are read (log_mfma.hip): clamping a code to [low, high] and
// subtracting low is exact in FP16, and 1 / (high - low) joins the output
// scale.
#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int HIST_T = 256;
constexpr int COPIES = 32;

// one workgroup of 256 per global copy
__global__ void zero_hist_kernel(int32_t* __restrict__ copies) {
    copies[blockIdx.x * 256 + threadIdx.x] = 0;
}

__global__ __launch_bounds__(HIST_T) void hist_kernel(const uint8_t* __restrict__ img, int h,
                                                      int w, long long pitch,
                                                      int32_t* __restrict__ copies,
                                                      int n_copies) {
    __shared__ uint32_t bins[256 * COPIES];  // bin b, copy c at b * COPIES + c
    for (int i = threadIdx.x; i < 256 * COPIES; i += HIST_T) bins[i] = 0u;
    __syncthreads();
    const int copy = threadIdx.x & (COPIES - 1);
    auto add4 = [&](uint32_t d) {
#pragma unroll
        for (int b = 0; b < 4; ++b) atomicAdd(&bins[((d >> (8 * b)) & 255u) * COPIES + copy], 1u);
    };
    const bool v16 = (pitch % 16 == 0) && (reinterpret_cast<uintptr_t>(img) % 16 == 0);
    const int w16 = v16 ? (w >> 4) : 0;
    for (int y = blockIdx.x; y < h; y += gridDim.x) {
        const uint8_t* row = img + static_cast<long long>(y) * pitch;
        for (int i = threadIdx.x; i < w16; i += HIST_T) {
            const uint4 d = reinterpret_cast<const uint4*>(row)[i];
            add4(d.x);
            add4(d.y);
            add4(d.z);
            add4(d.w);
        }
        for (int x = 16 * w16 + threadIdx.x; x < w; x += HIST_T)
            atomicAdd(&bins[row[x] * COPIES + copy], 1u);
    }
    __syncthreads();
    uint32_t n = 0;
#pragma unroll
    for (int c = 0; c < COPIES; ++c)  // rotated so the lanes read different banks
        n += bins[threadIdx.x * COPIES + ((c + threadIdx.x) & (COPIES - 1))];
    if (n) atomicAdd(&copies[(blockIdx.x % n_copies) * 256 + threadIdx.x], static_cast<int32_t>(n));
}

// levels[0] = low, levels[1] = high; hist (when not null) the summed bins.
__global__ __launch_bounds__(256) void levels_kernel(const int32_t* __restrict__ copies,
                                                     int n_copies, long long n_pixels,
                                                     int32_t* __restrict__ hist,
                                                     int32_t* __restrict__ levels) {
    __shared__ long long run[256];
    const int b = threadIdx.x;
    long long n = 0;
    for (int c = 0; c < n_copies; ++c) n += copies[c * 256 + b];
    if (hist) hist[b] = static_cast<int32_t>(n);  // at most h w < 2^31
    run[b] = n;
    __syncthreads();
    // inclusive scan from below (Hillis-Steele over 256 entries)
    for (int d = 1; d < 256; d <<= 1) {
        const long long t = b >= d ? run[b - d] : 0;
        __syncthreads();
        run[b] += t;
        __syncthreads();
    }
    const long long below = run[b];                           // pixels <= b
    const long long above = n_pixels - (b > 0 ? run[b - 1] : 0);  // pixels >= b
    const long long need = 175LL * n_pixels;
    const int short_low = __syncthreads_count(100000LL * below < need);
    const int short_high = __syncthreads_count(100000LL * above < need);
    if (b == 0) {
        levels[0] = short_low < 255 ? short_low : 255;
        levels[1] = 255 - (short_high < 255 ? short_high : 255);
    }
}

}  // namespace

// Workgroups of the histogram pass: up to two per CU with several global
// copies; with one copy, one per CU (fewer adds on each of its words).
int stretch_hist_blocks(int h, int n_cu, int n_copies) {
    const int cap = (n_copies > 1 ? 2 : 1) * (n_cu > 0 ? n_cu : 256);
    return h < cap ? h : cap;
}

hipError_t launch_stretch_levels(const uint8_t* img, int h, int w, long long pitch,
                                 int32_t* copies, int n_copies, int32_t* hist, int32_t* levels,
                                 int n_cu, hipStream_t s) {
    if (n_copies < 1 || n_copies > STRETCH_MAX_COPIES) return hipErrorInvalidValue;
    zero_hist_kernel<<<n_copies, 256, 0, s>>>(copies);
    hist_kernel<<<stretch_hist_blocks(h, n_cu, n_copies), HIST_T, 0, s>>>(img, h, w, pitch, copies,
                                                                         n_copies);
    levels_kernel<<<1, 256, 0, s>>>(copies, n_copies, static_cast<long long>(h) * w, hist, levels);
    return hipGetLastError();
}

}  // namespace mhfd
