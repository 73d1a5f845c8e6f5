// Scale-space operator on the matrix cores (u8 codes or fp32 values).
//
// The operator of one scale (the sigma^2-normalised Laplacian of the Gaussian
// of section 2.2, computed separably as in the strip kernel) is a pair of banded
// Toeplitz products, so it maps onto gfx950's 16x16x32 FP16 MFMA:
//
//   row pass     A = I * Tg, B = I * Th: M = 16 image rows, N = 16 output
//                columns, K = 32 input columns per instruction; the band of
//                2R + 1 taps spans ceil((16 + R + rw8) / 32) K-blocks, the
//                window starting rw8 = ceil8(R) columns left of the tile.
//   column pass  R = [A | B] * [Thc ; Tgc]: M = 16 columns, N = 16 output
//                rows, K = 32 intermediate rows per instruction; the window
//                starts R rows above the tile, ceil((16 + 2R) / 32) K-blocks.
//
// Precision.  u8 codes are exact in FP16; fp32 values are first scaled by an
// exact power of two that brings the tile's max |I| (a pre-pass) just below
// 2^14.  Every tap, fp32 input and intermediate is split into an FP16 pair
// hi + lo (hi = nearest FP16, lo = nearest FP16 of the exact FP32 remainder,
// error <= 2^-22 of the value), and each product is formed as hi*hi + hi*lo
// + lo*hi with FP32 accumulation (hi*hi + hi*lo for exact codes); the
// dropped lo*lo term is below 2^-22 of the product.  Powers of two scale the row taps so
// that intermediates stay below 2^15 and the column taps so that their largest
// entry is 2^14; values far below those maxima fall into FP16's subnormal
// range, where the absolute error (2^-25) is negligible against the maxima.
// The powers of two are undone exactly on the output.
//
// Data flow of one wave (no LDS, no barriers): the wave owns a 16-column tile
// and walks down a segment of rows.  It keeps its tap fragments in registers
// (they are the same for every tile of the scale) and a ring of the last
// 2 * NKC 16-row intermediate blocks.  The row-pass accumulator layout (lane
// = column, 4 consecutive rows per lane) is exactly the column pass's A
// operand once the K index of each 32-row block is permuted as
// {0..3, 16..19 | 4..7, 20..23 | ...}; the column taps are laid out with the
// same permutation, so intermediates never leave registers.
#include <math.h>
#include <stdint.h>

#include <vector>

#include <type_traits>

#include "mhfd_internal.h"

namespace mhfd {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int MW = MFMA_GROUP_WAVES;  // waves per workgroup, one 16-column tile each
constexpr int MAX_RADIUS = 56;  // largest radius with nkr, nkc <= 4

__device__ __forceinline__ float4_t mfma16(half8_t a, half8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Intermediate block: rows 4g..4g+3 of column c for lane (g, c), A and B as
// FP16 pairs.
struct Slot {
    half4_t ah, al, bh, bl;
};

// lo = the FP16 rounding of v - hi, formed as one mixed-precision FMA per
// value (hi * neg1 + v with hi read as FP16, rounded once), which is the
// rounding of the exact remainder.  neg1 = -1 arrives as an opaque register:
// with a literal -1 the product folds into a subtraction and the FMA is lost
// (two conversions and a subtraction per value).
__device__ __forceinline__ void split(float4_t v, half4_t& hi, half4_t& lo, float neg1) {
    hi = __builtin_convertvector(v, half4_t);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        lo[i] = static_cast<_Float16>(__builtin_fmaf(static_cast<float>(hi[i]), neg1, v[i]));
}

__device__ __forceinline__ half8_t cat(half4_t a, half4_t b) {
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Eight u8 codes (two dwords) -> FP16: each byte b becomes the FP16 bit
// pattern 0x64bb = 1024 + b, then 1024 is subtracted exactly.
__device__ __forceinline__ half8_t codes_plus_1024(uint32_t d0, uint32_t d1) {
    const uint32_t m = 0x64646464u;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    u4 q;
    q[0] = __builtin_amdgcn_perm(m, d0, 0x04010400u);
    q[1] = __builtin_amdgcn_perm(m, d0, 0x04030402u);
    q[2] = __builtin_amdgcn_perm(m, d1, 0x04010400u);
    q[3] = __builtin_amdgcn_perm(m, d1, 0x04030402u);
    return __builtin_bit_cast(half8_t, q);
}
__device__ __forceinline__ half8_t codes_to_half(uint32_t d0, uint32_t d1) {
    return codes_plus_1024(d0, d1) - static_cast<half8_t>(static_cast<_Float16>(1024.0f));
}

// One wave's work item: a 16-column tile from x0 over rows [y0, y1).  (Two
// tiles per wave would share the tap fragments and give more independent
// MFMA chains, but their rings push the large shapes past 256 VGPRs;
// measured on the 4096^2 workload one tile per wave is fastest.)
struct WaveJob {
    const void* img;  // u8 codes or fp32 values
    long long pitch;  // elements
    float* plane;     // output plane, row pitch w
    int h, w, x0, y0, y1, rw8, rwc;
    int aligned;      // rows aligned for whole 8-element group loads
    int out_vec;      // 16-byte aligned output rows and w % 4 == 0
    float in_scale;   // fp32 input: exact power of two applied before the split
    float neg1;       // -1, opaque to the compiler (split)
    float out_scale;  // exact power of two (times 255 / (high - low) when stretched)
    uint32_t s_lo, s_hi, s_nlo;  // stretched u8 input: 1024 + low, 1024 + high,
                                 // -(1024 + low), each as an FP16 pair
    // Threshold-sparse output (SPARSE kernels): the plane's activity words
    // (ceil(h/16) x act_bx) and the threshold.
    uint64_t* act;
    int act_bx;
    float tau;
    // Softplus-sum epilogue (EPI_SOFTSUM): the wave's sum of
    // softplus(sp_beta (|R| - sp_tau)) goes to *partial.
    double* partial;
    float sp_beta, sp_tau;
    // Cotangent epilogue (EPI_COTAN): r plane, sigma, w factor of the image.
    float* aux;
    float sigma, wb;
    uint32_t* cmax_word;
    // Second column-tap set (EPI_DUAL): output plane and factor.
    float* plane2;
    float out_scale2;
};

// 8-bit input with the histogram stretch applied as it is read (stretch.hip):
// codes clamped to [low, high], minus low.
struct U8Stretch {};
template <typename T>
struct Elem {
    typedef T type;
};
template <>
struct Elem<U8Stretch> {
    typedef uint8_t type;
};

// fp32 input: the scale that brings max |I| just below 2^14, from the bit
// pattern of max |I| (an exact power of two; 1 for zero or non-finite data,
// whose results are then unspecified).
__device__ __forceinline__ float input_scale(uint32_t maxbits) {
    const float m = __uint_as_float(maxbits);
    if (!(m > 0.0f) || !isfinite(m)) return 1.0f;
    int e;
    frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
    const int s = min(100, max(-120, 14 - e));
    return ldexpf(1.0f, s);
}

// Regular items (EDGE = false) read whole 8-element groups, store float4 rows
// and reflect rows and columns at most once.  Windows start on multiples of
// 8 columns, so when the width is a multiple of 8 every group lies wholly
// inside the image or wholly beyond one border; a group beyond a border is
// the mirrored group, loaded aligned and reversed.  The general form (EDGE =
// true: widths not a multiple of 8, tiles narrower than the window, partial
// 16-row or 16-column tiles) reflects every index as often as needed and
// guards every store.  Keeping the regular body free of the general code
// keeps its loop small and its memory waits exact.
// Input prefetch depth D (blocks of 16 rows loaded ahead of their row pass)
// and ring length NS (intermediate blocks held: at least the 2 nkc the
// column pass reads, rounded up to a multiple of D so that ring and prefetch
// slots repeat together).
// Measured on 4096^2 tiles: depth 4 with the peeled loop below pays for
// nkc = 1 (11% faster); for 8-bit inputs with nkc = 2, depth 4 (4 more
// registers per block of rows) is 4-5% faster than 2, for fp32 inputs 3%
// slower; for nkc = 3 depth 3 (ring unchanged) was no faster, and depth 4
// (ring of 8) spills.
template <typename T, int NKC>
constexpr int mfma_depth() {
    return NKC == 1 ? 4 : (NKC == 2 && sizeof(typename Elem<T>::type) == 1 ? 4 : 2);
}
// Whether the first ring turn is peeled off the main loop.
template <typename T, int NKC>
constexpr bool mfma_peel() { return NKC == 1; }
template <typename T, int NKC>
constexpr int mfma_ring() {
    return (2 * NKC + mfma_depth<T, NKC>() - 1) / mfma_depth<T, NKC>() * mfma_depth<T, NKC>();
}

template <typename T, int NKR, int NKC>
__device__ __forceinline__ bool regular_job(const WaveJob& J) {
    constexpr int NS = mfma_ring<T, NKC>(), D = mfma_depth<T, NKC>();
    const int xw = J.x0 - J.rw8;
    // rows touched: y0 - rwc ... y1 - rwc + 16 (NS - 1 + D) (ring and
    // prefetch overrun), reflected once at most
    // offsets formed with 24-bit multiplies: rows, widths and pitches below
    // 2^24, every input offset below 2^32 (output planes hold < 2^29 pixels)
    return J.aligned && J.out_vec && (J.w & 7) == 0 && J.x0 + 16 <= J.w && xw >= -J.w &&
           xw + 32 * NKR <= 2 * J.w && J.h >= J.rwc + 16 * (NS + D + 1) &&
           ((J.y1 - J.y0) & 15) == 0 && J.h < (1 << 24) && J.w < (1 << 24) &&
           J.pitch < (1 << 24) && static_cast<long long>(J.h) * J.pitch <= 0xFFFFFFFFLL;
}

// Input group of 8 elements per lane and K-block: the raw registers and
// their conversion to the MFMA operand(s).
template <typename T>
struct Input;

template <>
struct Input<uint8_t> {
    typedef uint2 Raw;  // 8 codes
    static constexpr int PRODUCTS = 2;  // code x (tap hi, tap lo): the code is exact
    __device__ static Raw load(const uint8_t* p) { return *reinterpret_cast<const uint2*>(p); }
    __device__ static Raw reverse(Raw v) {
        return make_uint2(__builtin_amdgcn_perm(0u, v.y, 0x00010203u),   // bswap
                          __builtin_amdgcn_perm(0u, v.x, 0x00010203u));
    }
    __device__ static Raw gather(const uint8_t* row, const int* col) {
        uint32_t d[2] = {0u, 0u};
#pragma unroll
        for (int i = 0; i < 8; ++i) d[i >> 2] |= static_cast<uint32_t>(row[col[i]]) << (8 * (i & 3));
        return make_uint2(d[0], d[1]);
    }
    __device__ static void convert(Raw v, const WaveJob&, half8_t& hi, half8_t&) {
        hi = codes_to_half(v.x, v.y);
    }
};

template <>
struct Input<U8Stretch> : Input<uint8_t> {
    // 1024 + v is exact in FP16, so are the clamp to [1024 + low, 1024 + high]
    // and the subtraction of 1024 + low
    __device__ static void convert(Raw v, const WaveJob& J, half8_t& hi, half8_t&) {
        // positive FP16 values order as their bit patterns: the clamp runs
        // on 16-bit integers (no NaN handling), the shift in FP16
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        typedef uint16_t us8 __attribute__((ext_vector_type(8)));
        const us8 lo8 = __builtin_bit_cast(us8, static_cast<u4>(J.s_lo));
        const us8 hi8 = __builtin_bit_cast(us8, static_cast<u4>(J.s_hi));
        const half8_t nlo8 = __builtin_bit_cast(half8_t, static_cast<u4>(J.s_nlo));
        const us8 q = __builtin_bit_cast(us8, codes_plus_1024(v.x, v.y));
        const us8 c = __builtin_elementwise_min(__builtin_elementwise_max(q, lo8), hi8);
        hi = __builtin_bit_cast(half8_t, c) + nlo8;
    }
};

template <>
struct Input<float> {
    struct Raw {
        float4_t a, b;
    };
    static constexpr int PRODUCTS = 3;  // hi x tap hi, hi x tap lo, lo x tap hi
    __device__ static Raw load(const float* p) {
        Raw r;
        r.a = *reinterpret_cast<const float4_t*>(p);
        r.b = *reinterpret_cast<const float4_t*>(p + 4);
        return r;
    }
    __device__ static Raw reverse(Raw v) {
        Raw r;
        r.a = __builtin_shufflevector(v.b, v.b, 3, 2, 1, 0);
        r.b = __builtin_shufflevector(v.a, v.a, 3, 2, 1, 0);
        return r;
    }
    __device__ static Raw gather(const float* row, const int* col) {
        Raw r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            r.a[i] = row[col[i]];
            r.b[i] = row[col[4 + i]];
        }
        return r;
    }
    __device__ static void convert(Raw v, const WaveJob& J, half8_t& hi, half8_t& lo) {
        half4_t h0, l0, h1, l1;
        split(v.a * J.in_scale, h0, l0, J.neg1);
        split(v.b * J.in_scale, h1, l1, J.neg1);
        hi = cat(h0, h1);
        lo = cat(l0, l1);
    }
};

template <typename T>
__device__ __forceinline__ typename Input<T>::Raw select_raw(bool c, typename Input<T>::Raw a,
                                                             typename Input<T>::Raw b);
template <>
__device__ __forceinline__ uint2 select_raw<uint8_t>(bool c, uint2 a, uint2 b) {
    return c ? a : b;
}
template <>
__device__ __forceinline__ uint2 select_raw<U8Stretch>(bool c, uint2 a, uint2 b) {
    return c ? a : b;
}
template <>
__device__ __forceinline__ Input<float>::Raw select_raw<float>(bool c, Input<float>::Raw a,
                                                               Input<float>::Raw b) {
    Input<float>::Raw r;
    r.a = c ? a.a : b.a;
    r.b = c ? a.b : b.b;
    return r;
}

// CTL: the column-pass tap fragments are read from LDS (`cl`, the block's
// copy) at every use instead of being held in registers.
// SPARSE: the stack is written only for the 4-pixel row groups that hold a
// value above J.tau, and every 16 x 16 output block's groups are marked in
// one activity word (bit 16 g + r: row r, columns 4 g ... 4 g + 3 of the
// block), which the maxima pass reads instead of the unwritten groups.
// INNER (regular jobs only): every row-pass window column lies inside the
// image, so no group is mirrored and the groups of a row are one base
// address plus constant offsets.
// EPI_DUAL: a second set of column taps (cl2, always in LDS) applied to the
// same ring, its result stored (dense) to J.plane2.
template <typename T, int NKR, int NKC, bool EDGE, bool CTL, bool SPARSE, int EPI = EPI_STORE,
          bool INNER = false>
__device__ __forceinline__ void wave_job(const WaveJob& J, const half8_t* __restrict__ fr,
                                         const half8_t* cl, int lane,
                                         const half8_t* cl2 = nullptr) {
    typedef Input<T> In;
    typedef typename In::Raw RawGroup;
    constexpr int NS = mfma_ring<T, NKC>();   // ring of intermediate blocks
    constexpr int D = mfma_depth<T, NKC>();   // input prefetch depth (divides NS)
    // Mirrored groups reversed at use rather than on arrival, so that the
    // wait for a load falls D blocks after it (costs registers: only with
    // the peeled loop or with the column taps in LDS).
    constexpr bool LATE_REV = mfma_peel<T, NKC>() || CTL;
    typedef typename Elem<T>::type E;
    const E* img = static_cast<const E*>(J.img);
    const int g = lane >> 4;
    const int c = lane & 15;
    const int h = J.h, w = J.w, x0 = J.x0, y0 = J.y0, y1 = J.y1;
    const int ntiles = (y1 - y0 + 15) >> 4;
    const int xw = x0 - J.rw8;  // first input column of the row-pass window
    const bool fast = !EDGE || (J.aligned && xw >= 0 && xw + 32 * NKR <= w);

    half8_t rt[NKR][4], ct[CTL ? 1 : NKC][4];
#pragma unroll
    for (int kb = 0; kb < NKR; ++kb)
#pragma unroll
        for (int t = 0; t < 4; ++t) rt[kb][t] = fr[(kb * 4 + t) * 64 + lane];
    if constexpr (!CTL) {
#pragma unroll
        for (int kb = 0; kb < NKC; ++kb)
#pragma unroll
            for (int t = 0; t < 4; ++t) ct[kb][t] = fr[((NKR + kb) * 4 + t) * 64 + lane];
    }

    // Regular items: source column and order of each 8-element group.
    int src[NKR];
    bool rev[NKR] = {};
    if (!EDGE && !INNER) {
#pragma unroll
        for (int kb = 0; kb < NKR; ++kb) {
            const int gs = xw + 32 * kb + 8 * g;
            rev[kb] = gs < 0 || gs >= w;
            src[kb] = gs < 0 ? -gs - 8 : (gs >= w ? 2 * w - 8 - gs : gs);
        }
    }
    // Raw input of intermediate block hb (image rows y0 - rwc + 16 hb ...):
    // one group per K-block and lane, loaded D blocks ahead of use.
    typedef RawGroup Raw[NKR];
    auto fetch = [&](int hb, Raw& raw) {
        const int yr = y0 - J.rwc + 16 * hb + c;
        int r;
        if (EDGE) {
            r = reflect_index(yr, h);
        } else {  // one reflection at most, without branches: -1 - yr = ~yr
            const int r0 = yr ^ (yr >> 31);
            r = min(r0, 2 * h - 1 - r0);
        }
        const E* row = EDGE ? img + static_cast<long long>(r) * J.pitch
                            : img + __umul24(static_cast<unsigned>(r),
                                             static_cast<unsigned>(J.pitch));
        if (INNER) {
            const E* base = row + xw + 8 * g;
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) raw[kb] = In::load(base + 32 * kb);
        } else if (!EDGE) {
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) {
                const RawGroup v = In::load(row + src[kb]);
                raw[kb] = LATE_REV ? v : select_raw<T>(rev[kb], In::reverse(v), v);
            }
        } else if (fast) {
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) raw[kb] = In::load(row + xw + 32 * kb + 8 * g);
        } else {
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) {
                int col[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) col[i] = reflect_index(xw + 32 * kb + 8 * g + i, w);
                raw[kb] = In::gather(row, col);
            }
        }
    };
    // Row pass of block hb from raw (then refilled with block hb + D).
    Raw raw[D];
    auto rowpass = [&](int hb, Raw& rw, Slot& out) {
        half8_t in_hi[NKR], in_lo[NKR];
#pragma unroll
        for (int kb = 0; kb < NKR; ++kb) {
            const RawGroup v = (EDGE || INNER || !LATE_REV)
                                   ? rw[kb]
                                   : select_raw<T>(rev[kb], In::reverse(rw[kb]), rw[kb]);
            In::convert(v, J, in_hi[kb], in_lo[kb]);
        }
        fetch(hb + D, rw);
        float4_t a = {0.f, 0.f, 0.f, 0.f}, b = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < NKR; ++kb) {
            a = mfma16(in_hi[kb], rt[kb][0], a);
            b = mfma16(in_hi[kb], rt[kb][2], b);
            a = mfma16(in_hi[kb], rt[kb][1], a);
            b = mfma16(in_hi[kb], rt[kb][3], b);
            if (In::PRODUCTS == 3) {
                a = mfma16(in_lo[kb], rt[kb][0], a);
                b = mfma16(in_lo[kb], rt[kb][2], b);
            }
        }
        split(a, out.ah, out.al, J.neg1);
        split(b, out.bh, out.bl, J.neg1);
    };

    const bool vec = !EDGE || (J.out_vec && x0 + 16 <= w);
    // element offset of (y, x0 + 4 g) in an output plane (regular jobs: a
    // full-rate 24-bit multiply instead of 64-bit arithmetic)
    auto opix = [&](int y) -> long long {
        if constexpr (EDGE)
            return static_cast<long long>(y) * w + x0 + 4 * g;
        else
            return __umul24(static_cast<unsigned>(y), static_cast<unsigned>(w)) +
                   static_cast<unsigned>(x0 + 4 * g);
    };
    // dense store of one output block row to `plane` (EPI_DUAL)
    auto put = [&](float* plane, int t, float4_t v) {
        const int y = y0 + 16 * t + c;
        if (EDGE && y >= y1) return;
        float* o = plane + opix(y);
        if (vec) {
            *reinterpret_cast<float4_t*>(o) = v;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x0 + 4 * g + i < w) o[i] = v[i];
        }
    };
    float tsum = 0.0f;  // EPI_SOFTSUM: this lane's softplus sum
    double gsum = 0.0;  // EPI_COTAN: this lane's sigma-gradient sum
    float cmx = 0.0f;   // EPI_COTAN: this lane's max |c|
    float cot_s2 = 0.0f, cot_2is = 0.0f;  // EPI_COTAN: sigma^2 and 2 / sigma
    if constexpr (EPI == EPI_COTAN) {
        cot_s2 = J.sigma * J.sigma;
        cot_2is = 2.0f / J.sigma;
    }
    // Inputs of the read-modify-write epilogues (EPI_COTAN: the D1 plane and
    // r; EPI_ACCUM: the plane), loaded when the block's step starts so that
    // the block's MFMA work covers their latency (vector rows only; the
    // general path reads them at the store).
    struct EpiIn {
        float4_t a, b;
    };
    auto epi_load = [&](int t) {
        EpiIn e{};
        if constexpr (EPI == EPI_COTAN || EPI == EPI_ACCUM) {
            const int y = y0 + 16 * t + c;
            if (vec && (!EDGE || y < y1)) {
                const long long at = opix(y);
                e.a = *reinterpret_cast<const float4_t*>(J.plane + at);
                if constexpr (EPI == EPI_COTAN) e.b = *reinterpret_cast<const float4_t*>(J.aux + at);
            }
        }
        return e;
    };
    auto store = [&](int t, float4_t v, const EpiIn& e) {
        const int y = y0 + 16 * t + c;
        if constexpr (EPI == EPI_COTAN) {
            if (EDGE && y >= y1) return;
            const long long at = opix(y);
            // Per value: w = wb sigmoid(z) sgn(r) (sigmoid through the hardware
            // exp and reciprocal, about 1 ulp each), the sigma partial
            // w (2 r / sigma + sigma^2 d) in FP32, summed over the lane's four
            // values and added to the FP64 sum once per block.  The partials'
            // inputs r and d carry FP32 rounding already, so FP64 arithmetic
            // per value (twice the issue cost) would add no accuracy.
            float part = 0.0f;
            auto one = [&](float dv, float& rv) {  // rv: r in, c out
                const float z = J.sp_beta * (fabsf(rv) - J.sp_tau);
                const float m = J.wb * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
                const float wv = rv > 0.0f ? m : (rv < 0.0f ? -m : 0.0f);
                part += wv * (cot_2is * rv + cot_s2 * dv);
                rv = wv * cot_s2;
                cmx = fmaxf(cmx, fabsf(rv));
            };
            if (vec) {
                const float4_t d1 = e.a;
                float4_t r = e.b;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float rv = r[i];
                    one(d1[i] + v[i], rv);
                    r[i] = rv;
                }
                *reinterpret_cast<float4_t*>(J.aux + at) = r;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (x0 + 4 * g + i < w) one(J.plane[at + i] + v[i], J.aux[at + i]);
            }
            gsum += static_cast<double>(part);
            return;
        }
        if constexpr (EPI == EPI_SOFTSUM) {
            // softplus(z) = max(z, 0) + log(1 + e^{-|z|}); the lane's four
            // log terms as one logarithm of their product (each factor in
            // (1, 2], the product at most 16): one hardware log2 instead of
            // four (quarter-rate instructions)
            if (!EDGE || y < y1) {
                float lin = 0.0f, prod = 1.0f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (!EDGE || x0 + 4 * g + i < w) {
                        const float z = J.sp_beta * (fabsf(v[i]) - J.sp_tau);
                        lin += fmaxf(z, 0.0f);
                        prod *= 1.0f + __expf(-fabsf(z));
                    }
                }
                tsum += lin + __logf(prod);
            }
            return;
        }
        if constexpr (SPARSE) {
            bool a = false;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a |= (!EDGE || x0 + 4 * g + i < w) && v[i] > J.tau;
            if (EDGE) a &= y < y1;
            const uint64_t m = __ballot(a);
            if (lane == 0) J.act[static_cast<long long>((y0 >> 4) + t) * J.act_bx + (x0 >> 4)] = m;
            if (!a) return;
        }
        if (EDGE && y >= y1) return;
        float* o = J.plane + opix(y);
        if constexpr (EPI == EPI_ACCUM) {  // o += v
            if (vec) {
                *reinterpret_cast<float4_t*>(o) = e.a + v;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (x0 + 4 * g + i < w) o[i] += v[i];
            }
            return;
        }
        if (!EDGE) {
            // Streaming store: the stack is read once, by the maxima pass, and
            // measured end to end it is faster when the stores do not stay
            // dirty in the caches that pass reads through.
            __builtin_nontemporal_store(v, reinterpret_cast<float4_t*>(o));
        } else if (vec) {
            *reinterpret_cast<float4_t*>(o) = v;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x0 + 4 * g + i < w) o[i] = v[i];
        }
    };

    Slot ring[NS];
#pragma unroll
    for (int q = 0; q < D; ++q) fetch(q, raw[q]);
#pragma unroll
    for (int p = 0; p < NS - 1; ++p) rowpass(p, raw[p % D], ring[p]);
    // Output block t at ring position p (= t mod NS).
    auto step = [&](int t, int p) {
        const EpiIn ein = epi_load(t);
        rowpass(t + NS - 1, raw[(p + NS - 1) % D], ring[(p + NS - 1) % NS]);
        float4_t ra = {0.f, 0.f, 0.f, 0.f}, rb = {0.f, 0.f, 0.f, 0.f};
        // LDS form: an opaque lane offset per block keeps the reads in the
        // loop (hoisted, they would be the registers this form saves)
        int lo = lane;
        if constexpr (CTL || EPI == EPI_DUAL) asm volatile("" : "+v"(lo));
        auto tap = [&](int kb, int t) -> half8_t {
            if constexpr (CTL)
                return cl[(kb * 4 + t) * 64 + lo];
            else
                return ct[kb][t];
        };
#pragma unroll
        for (int kb = 0; kb < NKC; ++kb) {
            const Slot& sa = ring[(p + 2 * kb) % NS];
            const Slot& sb = ring[(p + 2 * kb + 1) % NS];
            const half8_t xh = cat(sa.ah, sb.ah), xl = cat(sa.al, sb.al);
            const half8_t yh = cat(sa.bh, sb.bh), yl = cat(sa.bl, sb.bl);
            const half8_t c0 = tap(kb, 0), c2 = tap(kb, 2);
            ra = mfma16(xh, c0, ra);
            rb = mfma16(yh, c2, rb);
            ra = mfma16(xh, tap(kb, 1), ra);
            rb = mfma16(yh, tap(kb, 3), rb);
            ra = mfma16(xl, c0, ra);
            rb = mfma16(yl, c2, rb);
        }
        if constexpr (EPI == EPI_DUAL) {
            float4_t ra2 = {0.f, 0.f, 0.f, 0.f}, rb2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < NKC; ++kb) {
                const Slot& sa = ring[(p + 2 * kb) % NS];
                const Slot& sb = ring[(p + 2 * kb + 1) % NS];
                const half8_t xh = cat(sa.ah, sb.ah), xl = cat(sa.al, sb.al);
                const half8_t yh = cat(sa.bh, sb.bh), yl = cat(sa.bl, sb.bl);
                const half8_t d0 = cl2[(kb * 4 + 0) * 64 + lo], d2 = cl2[(kb * 4 + 2) * 64 + lo];
                ra2 = mfma16(xh, d0, ra2);
                rb2 = mfma16(yh, d2, rb2);
                ra2 = mfma16(xh, cl2[(kb * 4 + 1) * 64 + lo], ra2);
                rb2 = mfma16(yh, cl2[(kb * 4 + 3) * 64 + lo], rb2);
                ra2 = mfma16(xl, d0, ra2);
                rb2 = mfma16(yl, d2, rb2);
            }
            put(J.plane, t, (ra + rb) * J.out_scale);
            put(J.plane2, t, (ra2 + rb2) * J.out_scale2);
        } else {
            store(t, (ra + rb) * J.out_scale, ein);
        }
    };
    if constexpr (mfma_peel<T, NKC>()) {
        // Whole ring turns without exits, the first one peeled, then the
        // remaining blocks: the loop is entered with the same memory
        // operations in flight as at its back edge (loads of later rows, then
        // stores), so the waits at its head need only the prefetched rows,
        // not the last stores, to have landed.
        int t0 = 0;
        if (ntiles >= NS) {
#pragma unroll
            for (int p = 0; p < NS; ++p) step(p, p);
            for (t0 = NS; t0 + NS <= ntiles; t0 += NS) {
#pragma unroll
                for (int p = 0; p < NS; ++p) step(t0 + p, p);
            }
        }
#pragma unroll
        for (int p = 0; p < NS - 1; ++p)
            if (t0 + p < ntiles) step(t0 + p, p);
    } else {
        // one copy of the turn (register-bound shapes)
        for (int t0 = 0; t0 < ntiles; t0 += NS) {
#pragma unroll
            for (int p = 0; p < NS; ++p) {
                if (t0 + p >= ntiles) break;
                step(t0 + p, p);
            }
        }
    }
    if constexpr (EPI == EPI_SOFTSUM) {
        double t = tsum;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) *J.partial = t;
    }
    if constexpr (EPI == EPI_COTAN) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            gsum += __shfl_xor(gsum, o, 64);
            cmx = fmaxf(cmx, __shfl_xor(cmx, o, 64));
        }
        if (lane == 0) {
            *J.partial = gsum;
            if (cmx > 0.0f) atomicMax(J.cmax_word, __float_as_uint(cmx));
        }
    }
}

template <typename T, int NKR, int NKC, bool CTL = false, bool SPARSE = false, int EPI = EPI_STORE>
__device__ __forceinline__ void run_job(const WaveJob& J, const half8_t* __restrict__ fr,
                                        int lane, const half8_t* cl = nullptr,
                                        const half8_t* cl2 = nullptr) {
    if (regular_job<T, NKR, NKC>(J)) {
        const int xw = J.x0 - J.rw8;
        if (xw >= 0 && xw + 32 * NKR <= J.w)
            wave_job<T, NKR, NKC, false, CTL, SPARSE, EPI, true>(J, fr, cl, lane, cl2);
        else
            wave_job<T, NKR, NKC, false, CTL, SPARSE, EPI, false>(J, fr, cl, lane, cl2);
    } else {
        wave_job<T, NKR, NKC, true, CTL, SPARSE, EPI>(J, fr, cl, lane, cl2);
    }
}

// Kernels of shapes with nkc >= 3 read their column taps from LDS: the
// 4 nkc fragments (16 nkc KB per workgroup) would otherwise hold 16 nkc of
// the wave's registers.
template <int NKC>
constexpr bool mfma_cols_in_lds() { return NKC >= 3; }

// Two waves per SIMD where the live state fits 256 registers (u8: no spills
// up to nkc = 3; fp32 inputs carry twice the operands); otherwise one wave
// per SIMD.
template <typename T, int NKC>
constexpr int mfma_waves() { return NKC <= (sizeof(typename Elem<T>::type) == 1 ? 3 : 2) ? 2 : 1; }

// blockIdx.y: the image of a batch (L.img_stride, L.out_stride apart; fp32
// input: its own max |I| word maxbits[blockIdx.y]).
template <typename T, int NKR, int NKC, bool SPARSE, int EPI = EPI_STORE>
__global__ __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(mfma_waves<T, NKC>(), 2)))
void log_mfma_kernel(const typename Elem<T>::type* __restrict__ img, int h, int w,
                     long long pitch, int aligned, int out_vec,
                     const uint32_t* __restrict__ maxbits,
                     const half8_t* __restrict__ frags, MfmaLaunch L, float* __restrict__ out,
                     long long plane_stride, ActOut act) {
    const int bid = blockIdx.x;
    const int bimg = blockIdx.y;
    img += bimg * L.img_stride;
    out += bimg * L.out_stride;
    int si = 0;
    while (si + 1 < L.n && bid >= L.sc[si + 1].block_begin) ++si;
    const MfmaScale& sc = L.sc[si];
    const int local = bid - sc.block_begin;
    const int seg = local / L.groups_x;
    const int wcol = (local - seg * L.groups_x) * MW + (threadIdx.x >> 6);
    constexpr bool CTL = mfma_cols_in_lds<NKC>();
    constexpr bool DUAL = EPI == EPI_DUAL;
    __shared__ half8_t cl[CTL ? NKC * 4 * 64 : 1];
    __shared__ half8_t cl2[DUAL ? NKC * 4 * 64 : 1];
    if constexpr (CTL || DUAL) {  // the block's column fragments, before any wave leaves
        if constexpr (CTL) {
            const half8_t* src = frags + sc.frag_off + NKR * 4 * 64;
            for (int i = threadIdx.x; i < NKC * 4 * 64; i += 64 * MW) cl[i] = src[i];
        }
        if constexpr (DUAL) {
            const half8_t* src2 = frags + sc.frag_off2 + NKR * 4 * 64;
            for (int i = threadIdx.x; i < NKC * 4 * 64; i += 64 * MW) cl2[i] = src2[i];
        }
        __syncthreads();
    }
    // EPI_SOFTSUM, EPI_COTAN: one double per wave of the launch and image
    constexpr bool WAVE_SUM = EPI == EPI_SOFTSUM || EPI == EPI_COTAN;
    double* partial = nullptr;
    if constexpr (WAVE_SUM)
        partial = L.partial + (static_cast<long long>(bimg) * gridDim.x + bid) * MW + (threadIdx.x >> 6);
    if (wcol >= L.tiles_x) {
        if constexpr (WAVE_SUM)
            if ((threadIdx.x & 63) == 0) *partial = 0.0;
        return;
    }
    // fp32: maxbits = max |I| bits; stretched u8: maxbits = {low, high}
    float in_s = 1.0f, stretch = 1.0f;
    WaveJob J;
    J.neg1 = -1.0f;
    asm volatile("" : "+s"(J.neg1));
    J.s_lo = J.s_hi = 0x64006400u;
    J.s_nlo = 0xE400E400u;
    if constexpr (std::is_same<T, U8Stretch>::value) {
        // 1024 + c has FP16 bits 0x6400 + c for codes c in [0, 255]
        const int lo = static_cast<int>(maxbits[0]), hi = static_cast<int>(maxbits[1]);
        J.s_lo = (0x6400u + static_cast<uint32_t>(lo)) * 0x10001u;
        J.s_hi = (0x6400u + static_cast<uint32_t>(hi)) * 0x10001u;
        J.s_nlo = (0xE400u + static_cast<uint32_t>(lo)) * 0x10001u;  // sign bit set
        stretch = hi > lo ? 255.0f / static_cast<float>(hi - lo) : 0.0f;
    } else if (maxbits) {
        in_s = input_scale(maxbits[bimg]);
    }
    J.img = img;
    J.pitch = pitch;
    J.plane = out + static_cast<long long>(sc.plane) * plane_stride;
    J.h = h;
    J.w = w;
    J.x0 = wcol * 16;
    J.y0 = seg * sc.seg_rows;
    J.y1 = min(J.y0 + sc.seg_rows, h);
    J.rw8 = sc.rw8;
    J.rwc = sc.rwc;
    J.aligned = aligned;
    J.out_vec = out_vec;
    J.in_scale = in_s;
    J.out_scale = (L.dev_scale ? L.dev_scale[sc.dev_scale_idx] : sc.out_scale) / in_s * stretch;
    J.act = act.mask + static_cast<long long>(sc.plane) * act.by * act.bx;
    J.act_bx = act.bx;
    J.tau = act.tau;
    J.partial = partial;
    J.sp_beta = L.beta;
    J.sp_tau = L.tau;
    if constexpr (DUAL) {
        J.plane2 = L.aux + bimg * L.out_stride;
        J.out_scale2 = L.dev_scale[sc.dev_scale_idx2] / in_s;
    }
    if constexpr (EPI == EPI_COTAN) {
        J.aux = L.aux + bimg * L.out_stride;
        J.sigma = L.sigmas[L.soft_k];
        J.wb = static_cast<float>(static_cast<double>(L.gbar[bimg]) * L.inv_khw) * L.beta;
        J.cmax_word = L.cmax + bimg;
    }
    run_job<T, NKR, NKC, CTL, SPARSE, EPI>(J, frags + sc.frag_off, threadIdx.x & 63, cl, cl2);
}

// Persistent form over a batch of tiles: every workgroup pulls items (tile,
// scale j of the launch, row segment, group of MW adjacent wave columns) from
// a counter, and its waves run the single-tile path's per-wave body on them.
// Items are numbered tile-major, so the scales of a tile run together and
// re-read its image from the caches; for nkc >= 3 the scale's column taps
// sit in LDS as in the single-tile kernel, copied again when the scale
// changes.
template <typename T, int NKR, int NKC, bool SPARSE>
__global__ __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(mfma_waves<T, NKC>(), 2)))
void log_mfma_batch_kernel(int n_tiles, const BatchTile* __restrict__ tiles,
                           const uint32_t* __restrict__ maxbits, float* __restrict__ stack,
                           const half8_t* __restrict__ frags, MfmaBatchScales sc,
                           BatchCounters* __restrict__ ctr, int slot, uint64_t* act, float tau) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr bool CTL = mfma_cols_in_lds<NKC>();
    __shared__ half8_t cl[CTL ? NKC * 4 * 64 : 1];
    __shared__ int s_item;
    const int per_scale = ctr->mitems_per_scale;
    const int total = ctr->valid ? per_scale * sc.n : 0;
    int loaded = -1;  // scale whose column taps are in LDS (uniform)
    int lo = 0;       // tile of the last item (uniform)
    for (;;) {
        __syncthreads();  // every wave is done with s_item and the LDS taps
        if (threadIdx.x == 0) s_item = atomicAdd(&ctr->mwork[slot], 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar registers
        if (item >= total) break;
        // Tile-major: tile t owns items [S base_t, S base_t+1) (base: its
        // items per scale before it), scale-major inside, so the scales of
        // a tile run close together in time and re-read its image from the
        // caches rather than HBM.
        // The workgroup's items increase (one counter), so its tile only
        // moves forward: a cursor from the last item's tile.
        const int S = sc.n;
        while (lo + 1 < n_tiles && S * tiles[lo + 1].mitem_base <= item) ++lo;
        const BatchTile& t = tiles[lo];
        const int n_t = (lo + 1 < n_tiles ? tiles[lo + 1].mitem_base : per_scale) - t.mitem_base;
        const int r = item - S * t.mitem_base;
        const int j = r / n_t;
        if constexpr (CTL) {
            if (j != loaded) {
                const half8_t* src = frags + sc.frag_off[j] + NKR * 4 * 64;
                for (int i = threadIdx.x; i < NKC * 4 * 64; i += 64 * MW) cl[i] = src[i];
                __syncthreads();
                loaded = j;
            }
        }
        const int local = r - j * n_t;
        const int seg = local / t.mgroups_x;
        const int wcol = (local - seg * t.mgroups_x) * MW + wv;
        if (wcol >= t.mtiles_x) continue;
        const float in_s = maxbits ? input_scale(maxbits[lo]) : 1.0f;
        WaveJob J;
        J.neg1 = -1.0f;
        asm volatile("" : "+s"(J.neg1));
        J.img = t.img;
        J.pitch = t.pitch;
        J.h = t.h;
        J.w = t.w;
        J.plane = stack + t.stack_off + static_cast<long long>(sc.plane[j]) * t.h * t.w;
        J.x0 = wcol * 16;
        J.y0 = seg * t.mseg_rows;
        J.y1 = min(J.y0 + t.mseg_rows, t.h);
        J.rw8 = sc.rw8[j];
        J.rwc = sc.rwc[j];
        J.aligned = (t.pitch % 8 == 0) &&
                    (reinterpret_cast<uintptr_t>(t.img) % (8 * sizeof(T)) == 0);
        J.out_vec = (t.w % 4 == 0) && (t.stack_off % 4 == 0) &&
                    (reinterpret_cast<uintptr_t>(stack) % 16 == 0);
        J.in_scale = in_s;
        J.out_scale = sc.out_scale[j] / in_s;
        if constexpr (SPARSE) {
            J.act_bx = (t.w + 15) / 16;
            J.act = act + t.act_off + static_cast<long long>(sc.plane[j]) * ((t.h + 15) / 16) * J.act_bx;
            J.tau = tau;
        }
        run_job<T, NKR, NKC, CTL, SPARSE>(J, frags + sc.frag_off[j], lane, cl);
    }
}

// max |I| over rows [y, y+1) ... of an fp32 image: workgroups stride over
// rows, lanes over columns (float4 where rows are 16-byte aligned); no
// per-element division.
__device__ __forceinline__ float absmax4(float4_t v) {
    return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
}

// max |I| over rows row0, row0 + row_step, ... of an h x w fp32 image, the
// wave's lanes reduced.  Four rows are read per pass while four remain, so
// every lane keeps four loads in flight; then one row per pass.
__device__ __forceinline__ float rows_absmax(const float* __restrict__ img, int h, int w,
                                             long long pitch, int row0, int row_step) {
    const bool v4 = (pitch % 4 == 0) && (reinterpret_cast<uintptr_t>(img) % 16 == 0);
    const int w4 = v4 ? (w >> 2) : 0;
    float m = 0.0f;
    int y = row0;
    for (; y + 3 * row_step < h; y += 4 * row_step) {
        const float* r0 = img + static_cast<long long>(y) * pitch;
        const float* r1 = r0 + row_step * pitch;
        const float* r2 = r1 + row_step * pitch;
        const float* r3 = r2 + row_step * pitch;
        for (int i = threadIdx.x; i < w4; i += blockDim.x) {
            const float4_t a = reinterpret_cast<const float4_t*>(r0)[i];
            const float4_t b = reinterpret_cast<const float4_t*>(r1)[i];
            const float4_t c = reinterpret_cast<const float4_t*>(r2)[i];
            const float4_t d = reinterpret_cast<const float4_t*>(r3)[i];
            m = fmaxf(m, fmaxf(fmaxf(absmax4(a), absmax4(b)), fmaxf(absmax4(c), absmax4(d))));
        }
        for (int x = 4 * w4 + threadIdx.x; x < w; x += blockDim.x)
            m = fmaxf(m, fmaxf(fmaxf(fabsf(r0[x]), fabsf(r1[x])), fmaxf(fabsf(r2[x]), fabsf(r3[x]))));
    }
    for (; y < h; y += row_step) {
        const float* r0 = img + static_cast<long long>(y) * pitch;
        for (int i = threadIdx.x; i < w4; i += blockDim.x)
            m = fmaxf(m, absmax4(reinterpret_cast<const float4_t*>(r0)[i]));
        for (int x = 4 * w4 + threadIdx.x; x < w; x += blockDim.x) m = fmaxf(m, fabsf(r0[x]));
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
    return m;
}

// The workgroup's largest value (256 threads), valid in thread 0.  One
// atomic per workgroup: atomics on one word serialise, and one per wave
// made the pass several times slower than its loads.
__device__ __forceinline__ float block_max256(float m) {
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// max |I| of an fp32 image as float bits (non-negative floats order as their
// bit patterns), for the input scale.  `bits` must be zero on entry.
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ img, int h, int w,
                                                     long long pitch, uint32_t* __restrict__ bits) {
    const float m = block_max256(rows_absmax(img, h, w, pitch, blockIdx.x, gridDim.x));
    if (threadIdx.x == 0 && m > 0.0f) atomicMax(bits, __float_as_uint(m));
}

// Per-tile max |I| of a batch (bits[t] zero on entry): workgroup row y of
// the grid takes tile y, and the gridDim.x workgroups of that row split its
// rows.
__global__ __launch_bounds__(256) void absmax_batch_kernel(const BatchTile* __restrict__ tiles,
                                                           const BatchCounters* __restrict__ ctr,
                                                           uint32_t* __restrict__ bits) {
    if (!ctr->valid) return;
    const int t = blockIdx.y;
    const BatchTile& d = tiles[t];
    const float m = block_max256(rows_absmax(static_cast<const float*>(d.img), d.h, d.w, d.pitch,
                                             blockIdx.x, gridDim.x));
    if (threadIdx.x == 0 && m > 0.0f) atomicMax(bits + t, __float_as_uint(m));
}

__global__ void zero_words_kernel(uint32_t* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename T, int NKR, int NKC>
hipError_t launch_one(const typename Elem<T>::type* img, int h, int w, int64_t pitch,
                      const uint32_t* maxbits,
                      const uint16_t* frags, const MfmaLaunch& L, float* out,
                      long long plane_stride, const ActOut& act, hipStream_t s) {
    int blocks = 0;
    for (int i = 0; i < L.n; ++i) blocks += L.sc[i].n_blocks;
    if (blocks == 0) return hipSuccess;
    const int aligned =
        (pitch % 8 == 0) &&
        (reinterpret_cast<uintptr_t>(img) % (8 * sizeof(typename Elem<T>::type)) == 0);
    // float4 stores need 16-byte aligned rows and planes
    const int out_vec = (w % 4 == 0) && (plane_stride % 4 == 0) &&
                        (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    if (act.mask)
        log_mfma_kernel<T, NKR, NKC, true><<<blocks, 64 * MW, 0, s>>>(
            img, h, w, static_cast<long long>(pitch), aligned, out_vec, maxbits,
            reinterpret_cast<const half8_t*>(frags), L, out, plane_stride, act);
    else
        log_mfma_kernel<T, NKR, NKC, false><<<blocks, 64 * MW, 0, s>>>(
            img, h, w, static_cast<long long>(pitch), aligned, out_vec, maxbits,
            reinterpret_cast<const half8_t*>(frags), L, out, plane_stride, act);
    return hipGetLastError();
}

// FP16 bit pattern nearest to x (ties to even); |x| < 65520.
uint16_t half_bits(double x) {
    uint16_t sign = 0;
    if (x < 0) {
        sign = 0x8000;
        x = -x;
    }
    if (x == 0.0) return sign;
    int e2;
    frexp(x, &e2);
    int E = e2 - 1;  // x = 1.f * 2^E
    if (E < -14) {
        const double q = nearbyint(ldexp(x, 24));  // subnormal quantum 2^-24
        return static_cast<uint16_t>(sign | static_cast<uint16_t>(q));
    }
    double q = nearbyint(ldexp(x, 10 - E));  // in [1024, 2048]
    if (q >= 2048.0) {
        q = 1024.0;
        ++E;
    }
    return static_cast<uint16_t>(sign | ((E + 15) << 10) | (static_cast<int>(q) - 1024));
}

double half_value(uint16_t b) {
    const double s = (b & 0x8000) ? -1.0 : 1.0;
    const int e = (b >> 10) & 31;
    const int f = b & 1023;
    if (e == 0) return s * ldexp(f, -24);
    return s * ldexp(1024 + f, e - 25);
}

// Largest integer S with m * 2^S <= limit (m > 0).
int pow2_fit(double m, double limit) {
    int S = static_cast<int>(floor(log2(limit / m)));
    while (ldexp(m, S + 1) <= limit) ++S;
    while (ldexp(m, S) > limit) --S;
    return S;
}

}  // namespace

bool mfma_radius_ok(int radius) { return radius >= 0 && radius <= MAX_RADIUS; }

MfmaShape mfma_shape(int radius) {
    MfmaShape s;
    s.rw8 = (radius + 7) / 8 * 8;
    if (s.rw8 < 8) s.rw8 = 8;
    // The ring's 16-row grid may start anywhere, so the column window starts
    // exactly R rows above the tile and spans 16 + 2R rows.
    s.rwc = radius;
    s.nkr = (16 + radius + s.rw8 + 31) / 32;
    s.nkc = (16 + 2 * radius + 31) / 32;
    return s;
}

size_t mfma_frag_halves(int radius) {
    const MfmaShape s = mfma_shape(radius);
    return static_cast<size_t>(s.nkr + s.nkc) * 4 * 64 * 8;
}

float mfma_build_frags(const double* g, const double* h, int R, double norm, double in_scale,
                       double in_max, uint16_t* dst) {
    const MfmaShape s = mfma_shape(R);
    std::vector<double> tg(R + 1), th(R + 1);
    double sg = 0.0, sh = 0.0;
    for (int j = 0; j <= R; ++j) {
        tg[j] = g[j] / in_scale;
        th[j] = h[j] / in_scale;
        sg += (j ? 2.0 : 1.0) * fabs(tg[j]);
        sh += (j ? 2.0 : 1.0) * fabs(th[j]);
    }
    // Row taps: intermediates in_max * sum |t| * 2^S stay at or below 2^15.
    const int Sg = pow2_fit(in_max * sg, 32768.0);
    const int Sh = sh > 0.0 ? pow2_fit(in_max * sh, 32768.0) : 0;
    std::vector<double> ca(R + 1), cb(R + 1);
    double cmax = 0.0;
    for (int j = 0; j <= R; ++j) {
        ca[j] = norm * h[j] * ldexp(1.0, -Sg);
        cb[j] = norm * g[j] * ldexp(1.0, -Sh);
        cmax = fmax(cmax, fmax(fabs(ca[j]), fabs(cb[j])));
    }
    // Column taps: largest entry at most 2^14.
    const int Sc = pow2_fit(cmax, 16384.0);
    auto emit = [&](double v, int part) {
        const uint16_t hi = half_bits(v);
        return part == 0 ? hi : half_bits(v - half_value(hi));
    };
    uint16_t* d = dst;
    for (int kb = 0; kb < s.nkr; ++kb)
        for (int t = 0; t < 4; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int n = lane & 15, gq = lane >> 4;
                    const int j = 32 * kb + 8 * gq + i - s.rw8 - n;
                    const int a = j < 0 ? -j : j;
                    double v = 0.0;
                    if (a <= R) v = (t < 2 ? ldexp(tg[a], Sg) : ldexp(th[a], Sh));
                    *d++ = emit(v, t & 1);
                }
    for (int kb = 0; kb < s.nkc; ++kb)
        for (int t = 0; t < 4; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int n = lane & 15, gq = lane >> 4;
                    const int r = 32 * kb + (i < 4 ? 4 * gq + i : 16 + 4 * gq + (i - 4));
                    const int j = r - s.rwc - n;
                    const int a = j < 0 ? -j : j;
                    double v = 0.0;
                    if (a <= R) v = ldexp(t < 2 ? ca[a] : cb[a], Sc);
                    *d++ = emit(v, t & 1);
                }
    return static_cast<float>(ldexp(1.0, -Sc));
}

int mfma_wave_tiles(int w) { return (w + MFMA_WAVE_COLS - 1) / MFMA_WAVE_COLS; }
int mfma_waves_per_block() { return MW; }

hipError_t launch_log_mfma_batch(int in_dtype, int nkr, int nkc, int n_tiles,
                                 const BatchTile* tiles, const uint32_t* maxbits, float* stack,
                                 const uint16_t* frags, const MfmaBatchScales& sc,
                                 BatchCounters* ctr, int slot, int grid, uint64_t* act, float tau,
                                 hipStream_t s) {
    if (sc.n == 0) return hipSuccess;
    const half8_t* f = reinterpret_cast<const half8_t*>(frags);
#define MHFD_MFMA_BATCH_CASE(T, A)                                                            \
    if (nkr == A && nkc == A) {                                                               \
        if (act)                                                                              \
            log_mfma_batch_kernel<T, A, A, true><<<grid, 64 * MW, 0, s>>>(                    \
                n_tiles, tiles, maxbits, stack, f, sc, ctr, slot, act, tau);                  \
        else                                                                                  \
            log_mfma_batch_kernel<T, A, A, false><<<grid, 64 * MW, 0, s>>>(                   \
                n_tiles, tiles, maxbits, stack, f, sc, ctr, slot, act, tau);                  \
        return hipGetLastError();                                                             \
    }
    if (in_dtype == MHFD_U8) {
        MHFD_MFMA_BATCH_CASE(uint8_t, 1)
        MHFD_MFMA_BATCH_CASE(uint8_t, 2)
        MHFD_MFMA_BATCH_CASE(uint8_t, 3)
        MHFD_MFMA_BATCH_CASE(uint8_t, 4)
    } else {
        MHFD_MFMA_BATCH_CASE(float, 1)
        MHFD_MFMA_BATCH_CASE(float, 2)
        MHFD_MFMA_BATCH_CASE(float, 3)
        MHFD_MFMA_BATCH_CASE(float, 4)
    }
#undef MHFD_MFMA_BATCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_log_mfma(int in_dtype, int stretch, int nkr, int nkc, const void* img, int h,
                           int w, int64_t pitch, const uint32_t* maxbits, const uint16_t* frags,
                           const MfmaLaunch& L, float* out, long long plane_stride,
                           const ActOut& act, hipStream_t s) {
#define MHFD_MFMA_CASE(T, A)                                                                \
    if (nkr == A && nkc == A)                                                               \
        return launch_one<T, A, A>(static_cast<const typename Elem<T>::type*>(img), h, w,   \
                                   pitch, maxbits, frags, L, out, plane_stride, act, s);
    if (in_dtype == MHFD_U8 && stretch) {
        MHFD_MFMA_CASE(U8Stretch, 1)
        MHFD_MFMA_CASE(U8Stretch, 2)
        MHFD_MFMA_CASE(U8Stretch, 3)
        MHFD_MFMA_CASE(U8Stretch, 4)
    } else if (in_dtype == MHFD_U8) {
        MHFD_MFMA_CASE(uint8_t, 1)
        MHFD_MFMA_CASE(uint8_t, 2)
        MHFD_MFMA_CASE(uint8_t, 3)
        MHFD_MFMA_CASE(uint8_t, 4)
    } else {
        MHFD_MFMA_CASE(float, 1)
        MHFD_MFMA_CASE(float, 2)
        MHFD_MFMA_CASE(float, 3)
        MHFD_MFMA_CASE(float, 4)
    }
#undef MHFD_MFMA_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_log_mfma_soft(int epi, int nkr, int nkc, const float* img, int h, int w,
                                int batch, const uint32_t* maxbits, const uint16_t* frags,
                                const MfmaLaunch& L, float* out, hipStream_t s) {
    int blocks = 0;
    for (int i = 0; i < L.n; ++i) blocks += L.sc[i].n_blocks;
    if (blocks == 0 || batch == 0) return hipSuccess;
    const int aligned = (w % 8 == 0) && (reinterpret_cast<uintptr_t>(img) % 32 == 0) &&
                        (L.img_stride % 8 == 0);
    const int out_vec = (w % 4 == 0) && (L.out_stride % 4 == 0) &&
                        (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    const half8_t* f = reinterpret_cast<const half8_t*>(frags);
    const dim3 grid(blocks, batch);
    if (epi == EPI_COTAN) zero_words_kernel<<<(batch + 255) / 256, 256, 0, s>>>(L.cmax, batch);
#define MHFD_SOFT_CASE(A, E)                                                                  \
    if (nkr == A && nkc == A && epi == E) {                                                   \
        log_mfma_kernel<float, A, A, false, E><<<grid, 64 * MW, 0, s>>>(                      \
            img, h, w, static_cast<long long>(w), aligned, out_vec, maxbits, f, L, out, 0,    \
            ActOut{nullptr, 0, 0, 0.0f});                                                     \
        return hipGetLastError();                                                             \
    }
#define MHFD_SOFT_SHAPE(A)         \
    MHFD_SOFT_CASE(A, EPI_STORE)   \
    MHFD_SOFT_CASE(A, EPI_ACCUM)   \
    MHFD_SOFT_CASE(A, EPI_SOFTSUM) \
    MHFD_SOFT_CASE(A, EPI_COTAN)   \
    MHFD_SOFT_CASE(A, EPI_DUAL)
    MHFD_SOFT_SHAPE(1)
    MHFD_SOFT_SHAPE(2)
    MHFD_SOFT_SHAPE(3)
    MHFD_SOFT_SHAPE(4)
#undef MHFD_SOFT_SHAPE
#undef MHFD_SOFT_CASE
    return hipErrorInvalidValue;
}

// max |I| of each image of a batch of b dense h x w fp32 images (bits[i]).
__global__ __launch_bounds__(256) void absmax_images_kernel(const float* __restrict__ imgs, int h,
                                                            int w, uint32_t* __restrict__ bits) {
    const int b = blockIdx.y;
    const float m = block_max256(rows_absmax(imgs + static_cast<long long>(b) * h * w, h, w,
                                             static_cast<long long>(w), blockIdx.x, gridDim.x));
    if (threadIdx.x == 0 && m > 0.0f) atomicMax(bits + b, __float_as_uint(m));
}

hipError_t launch_absmax_images(const float* imgs, int batch, int h, int w, uint32_t* bits,
                                hipStream_t s) {
    zero_words_kernel<<<(batch + 255) / 256, 256, 0, s>>>(bits, batch);
    const int blocks = (h + 3) / 4 < 128 ? (h + 3) / 4 : 128;
    absmax_images_kernel<<<dim3(blocks, batch), 256, 0, s>>>(imgs, h, w, bits);
    return hipGetLastError();
}

hipError_t launch_absmax(const float* img, int h, int w, int64_t pitch, uint32_t* bits,
                         hipStream_t s) {
    zero_words_kernel<<<1, 64, 0, s>>>(bits, 1);
    // a workgroup per four rows, up to 512 workgroups
    const int blocks = (h + 3) / 4 < 512 ? (h + 3) / 4 : 512;
    absmax_kernel<<<blocks, 256, 0, s>>>(img, h, w, static_cast<long long>(pitch), bits);
    return hipGetLastError();
}

hipError_t launch_absmax_batch(int n_tiles, const BatchTile* tiles, const BatchCounters* ctr,
                               uint32_t* bits, int grid, hipStream_t s) {
    zero_words_kernel<<<(n_tiles + 255) / 256, 256, 0, s>>>(bits, n_tiles);
    const int per_tile = grid / n_tiles > 4 ? grid / n_tiles : 4;
    absmax_batch_kernel<<<dim3(per_tile, n_tiles), 256, 0, s>>>(tiles, ctr, bits);
    return hipGetLastError();
}

}  // namespace mhfd
