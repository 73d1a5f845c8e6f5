// Scale-space operator of u8 tiles on the matrix cores.
//
// The operator of one scale (the sigma^2-normalised Laplacian of the Gaussian
// of section 3, computed separably as in the strip kernel) is a pair of banded
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
// Precision.  u8 codes are exact in FP16.  Every tap and every intermediate is
// split into an FP16 pair hi + lo (hi = nearest FP16, lo = nearest FP16 of the
// exact FP32 remainder, error <= 2^-22 of the value), and each product is
// formed as hi*hi + hi*lo + lo*hi with FP32 accumulation; the dropped lo*lo
// term is below 2^-22 of the product.  Powers of two scale the row taps so
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

#include "mhfd_internal.h"

namespace mhfd {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int MW = 4;          // waves per workgroup, one 16-column tile each
constexpr int MAX_RADIUS = 56;  // largest radius with nkr, nkc <= 4

__device__ __forceinline__ float4_t mfma16(half8_t a, half8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Intermediate block: rows 4g..4g+3 of column c for lane (g, c), A and B as
// FP16 pairs.
struct Slot {
    half4_t ah, al, bh, bl;
};

__device__ __forceinline__ void split(float4_t v, half4_t& hi, half4_t& lo) {
    hi = __builtin_convertvector(v, half4_t);
    const float4_t r = v - __builtin_convertvector(hi, float4_t);  // exact in FP32
    lo = __builtin_convertvector(r, half4_t);
}

__device__ __forceinline__ half8_t cat(half4_t a, half4_t b) {
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Eight u8 codes (two dwords) -> FP16: each byte b becomes the FP16 bit
// pattern 0x64bb = 1024 + b, then 1024 is subtracted exactly.
__device__ __forceinline__ half8_t codes_to_half(uint32_t d0, uint32_t d1) {
    const uint32_t m = 0x64646464u;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    u4 q;
    q[0] = __builtin_amdgcn_perm(m, d0, 0x04010400u);
    q[1] = __builtin_amdgcn_perm(m, d0, 0x04030402u);
    q[2] = __builtin_amdgcn_perm(m, d1, 0x04010400u);
    q[3] = __builtin_amdgcn_perm(m, d1, 0x04030402u);
    half8_t v = __builtin_bit_cast(half8_t, q);
    return v - static_cast<half8_t>(static_cast<_Float16>(1024.0f));
}

// One wave's work item: WT adjacent 16-column tiles from x0 over rows
// [y0, y1).  Several tiles per wave would share the tap fragments and give
// more independent MFMA chains, but their rings push the large shapes past
// 256 VGPRs; measured on the 4096^2 workload one tile per wave is fastest.
constexpr int WT = 1;
static_assert(16 * WT == MFMA_WAVE_COLS, "wave width");

struct WaveJob {
    const uint8_t* img;
    long long pitch;
    float* plane;     // output plane, row pitch w
    int h, w, x0, y0, y1, rw8, rwc;
    int aligned;      // 8-byte aligned rows: vector loads allowed in the interior
    int out_vec;      // 16-byte aligned output rows and w % 4 == 0
    float out_scale;
};

// Regular items (EDGE = false) read whole 8-byte groups, store float4 rows
// and reflect rows and columns at most once.  Windows start on multiples of
// 8 columns, so when the width is a multiple of 8 every 8-byte group lies
// wholly inside the image or wholly beyond one border; a group beyond a
// border is the mirrored group, loaded aligned and byte-reversed.  The
// general form (EDGE = true: widths not a multiple of 8, tiles narrower than
// the window, partial 16-row or 16-column tiles) reflects every index as
// often as needed and guards every store.  Keeping the regular body free of
// the general code keeps its loop small and its memory waits exact.
template <int NKR, int NKC, int NT>
__device__ __forceinline__ bool regular_job(const WaveJob& J) {
    constexpr int NS = 2 * NKC;
    const int xw = J.x0 - J.rw8;
    // rows touched: y0 - rwc ... y1 + 16 (NS + 2) (prefetch overrun)
    return J.aligned && J.out_vec && (J.w & 7) == 0 && J.x0 + 16 * NT <= J.w && xw >= -J.w &&
           xw + 16 * (NT - 1) + 32 * NKR <= 2 * J.w && J.h >= J.rwc + 16 * (NS + 3) &&
           ((J.y1 - J.y0) & 15) == 0;
}

template <int NKR, int NKC, int NT, bool EDGE>
__device__ __forceinline__ void wave_job(const WaveJob& J, const half8_t* __restrict__ fr,
                                         int lane) {
    constexpr int NS = 2 * NKC;        // ring of intermediate blocks
    constexpr int D = 2;  // input prefetch depth (divides NS)
    const int g = lane >> 4;
    const int c = lane & 15;
    const int h = J.h, w = J.w, x0 = J.x0, y0 = J.y0, y1 = J.y1;
    const int ntiles = (y1 - y0 + 15) >> 4;
    const int xw = x0 - J.rw8;  // first input column of the row-pass window
    const bool fast = !EDGE || (J.aligned && xw >= 0 && xw + 32 * NKR <= w);

    half8_t rt[NKR][4], ct[NKC][4];
#pragma unroll
    for (int kb = 0; kb < NKR; ++kb)
#pragma unroll
        for (int t = 0; t < 4; ++t) rt[kb][t] = fr[(kb * 4 + t) * 64 + lane];
#pragma unroll
    for (int kb = 0; kb < NKC; ++kb)
#pragma unroll
        for (int t = 0; t < 4; ++t) ct[kb][t] = fr[((NKR + kb) * 4 + t) * 64 + lane];

    // Regular items: source column and byte order of each 8-byte group.
    int src[NT][NKR];
    bool rev[NT][NKR];
    if (!EDGE) {
#pragma unroll
        for (int s = 0; s < NT; ++s)
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) {
                const int gs = xw + 16 * s + 32 * kb + 8 * g;
                rev[s][kb] = gs < 0 || gs >= w;
                src[s][kb] = gs < 0 ? -gs - 8 : (gs >= w ? 2 * w - 8 - gs : gs);
            }
    }
    // Raw codes of intermediate block hb (image rows y0 - rwc + 16 hb ...):
    // NKR pairs of dwords per lane and tile, loaded D blocks ahead of use.
    typedef uint2 Raw[NT][NKR];
    auto fetch = [&](int hb, Raw& raw) {
        const int yr = y0 - J.rwc + 16 * hb + c;
        int r;
        if (EDGE) {
            r = reflect_index(yr, h);
        } else {  // one reflection at most, without branches: -1 - yr = ~yr
            const int r0 = yr ^ (yr >> 31);
            r = min(r0, 2 * h - 1 - r0);
        }
        const uint8_t* row = J.img + static_cast<long long>(r) * J.pitch;
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            if (!EDGE) {
#pragma unroll
                for (int kb = 0; kb < NKR; ++kb) {
                    const uint2 v = *reinterpret_cast<const uint2*>(row + src[s][kb]);
                    const uint32_t lo = __builtin_amdgcn_perm(0u, v.y, 0x00010203u);  // bswap
                    const uint32_t hi = __builtin_amdgcn_perm(0u, v.x, 0x00010203u);
                    raw[s][kb] = rev[s][kb] ? make_uint2(lo, hi) : v;
                }
            } else if (fast) {
#pragma unroll
                for (int kb = 0; kb < NKR; ++kb)
                    raw[s][kb] = *reinterpret_cast<const uint2*>(row + xw + 32 * kb + 8 * g);
            } else {
#pragma unroll
                for (int kb = 0; kb < NKR; ++kb) {
                    uint32_t d[2] = {0u, 0u};
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int col = reflect_index(xw + 32 * kb + 8 * g + i, w);
                        d[i >> 2] |= static_cast<uint32_t>(row[col]) << (8 * (i & 3));
                    }
                    raw[s][kb] = make_uint2(d[0], d[1]);
                }
            }
        }
    };
    // Row pass of block hb from raw (then refilled with block hb + D).
    Raw raw[D];
    auto rowpass = [&](int hb, Raw& rw, Slot (&out)[NT]) {
        half8_t in[NT][NKR];
#pragma unroll
        for (int s = 0; s < NT; ++s)
#pragma unroll
            for (int kb = 0; kb < NKR; ++kb) in[s][kb] = codes_to_half(rw[s][kb].x, rw[s][kb].y);
        fetch(hb + D, rw);
        float4_t a[NT], b[NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) a[s] = b[s] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < NKR; ++kb)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int s = 0; s < NT; ++s) {
                    a[s] = mfma16(in[s][kb], rt[kb][q], a[s]);
                    b[s] = mfma16(in[s][kb], rt[kb][2 + q], b[s]);
                }
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            split(a[s], out[s].ah, out[s].al);
            split(b[s], out[s].bh, out[s].bl);
        }
    };

    const bool vec = !EDGE || (J.out_vec && x0 + 16 <= w);
    auto store = [&](int t, int s, float4_t v) {
        const int y = y0 + 16 * t + c;
        if (EDGE && y >= y1) return;
        float* o = J.plane + static_cast<long long>(y) * w + x0 + 16 * s + 4 * g;
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

    Slot ring[NS][NT];
#pragma unroll
    for (int q = 0; q < D; ++q) fetch(q, raw[q]);
#pragma unroll
    for (int p = 0; p < NS - 1; ++p) rowpass(p, raw[p % D], ring[p]);
    for (int t0 = 0; t0 < ntiles; t0 += NS) {
#pragma unroll
        for (int p = 0; p < NS; ++p) {
            const int t = t0 + p;
            if (t >= ntiles) break;
            rowpass(t + NS - 1, raw[(p + NS - 1) % D], ring[(p + NS - 1) % NS]);
            float4_t ra[NT], rb[NT];
#pragma unroll
            for (int s = 0; s < NT; ++s) ra[s] = rb[s] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < NKC; ++kb)
#pragma unroll
                for (int s = 0; s < NT; ++s) {
                    const Slot& sa = ring[(p + 2 * kb) % NS][s];
                    const Slot& sb = ring[(p + 2 * kb + 1) % NS][s];
                    const half8_t xh = cat(sa.ah, sb.ah), xl = cat(sa.al, sb.al);
                    const half8_t yh = cat(sa.bh, sb.bh), yl = cat(sa.bl, sb.bl);
                    ra[s] = mfma16(xh, ct[kb][0], ra[s]);
                    rb[s] = mfma16(yh, ct[kb][2], rb[s]);
                    ra[s] = mfma16(xh, ct[kb][1], ra[s]);
                    rb[s] = mfma16(yh, ct[kb][3], rb[s]);
                    ra[s] = mfma16(xl, ct[kb][0], ra[s]);
                    rb[s] = mfma16(yl, ct[kb][2], rb[s]);
                }
#pragma unroll
            for (int s = 0; s < NT; ++s) store(t, s, (ra[s] + rb[s]) * J.out_scale);
        }
    }
}

// A wave's job: both tiles through the regular body, or each existing tile
// through the general one.
template <int NKR, int NKC>
__device__ __forceinline__ void run_job(WaveJob J, const half8_t* __restrict__ fr, int lane) {
    if (regular_job<NKR, NKC, WT>(J)) {
        wave_job<NKR, NKC, WT, false>(J, fr, lane);
        return;
    }
    const int x0 = J.x0;
    for (int s = 0; s < WT; ++s) {
        J.x0 = x0 + 16 * s;
        if (J.x0 >= J.w) break;
        wave_job<NKR, NKC, 1, true>(J, fr, lane);
    }
}

// Two waves per SIMD where the live state fits 256 registers (no spills up
// to nkc = 3 in the single-tile kernel, nkc = 2 in the persistent one, whose
// item loop keeps more state); otherwise one wave per SIMD.
template <int NKC>
constexpr int mfma_waves() { return NKC <= 3 ? 2 : 1; }
template <int NKC>
constexpr int mfma_batch_waves() { return NKC <= 2 ? 2 : 1; }

template <int NKR, int NKC>
__global__ __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(mfma_waves<NKC>(), 2)))
void log_mfma_u8_kernel(
    const uint8_t* __restrict__ img, int h, int w, long long pitch, int aligned, int out_vec,
    const half8_t* __restrict__ frags, MfmaLaunch L, float* __restrict__ out,
    long long plane_stride) {
    const int bid = blockIdx.x;
    int si = 0;
    while (si + 1 < L.n && bid >= L.sc[si + 1].block_begin) ++si;
    const MfmaScale& sc = L.sc[si];
    const int local = bid - sc.block_begin;
    const int seg = local / L.groups_x;
    const int wcol = (local - seg * L.groups_x) * MW + (threadIdx.x >> 6);
    if (wcol >= L.tiles_x) return;
    WaveJob J;
    J.img = img;
    J.pitch = pitch;
    J.plane = out + static_cast<long long>(sc.plane) * plane_stride;
    J.h = h;
    J.w = w;
    J.x0 = wcol * 16 * WT;
    J.y0 = seg * sc.seg_rows;
    J.y1 = min(J.y0 + sc.seg_rows, h);
    J.rw8 = sc.rw8;
    J.rwc = sc.rwc;
    J.aligned = aligned;
    J.out_vec = out_vec;
    J.out_scale = sc.out_scale;
    run_job<NKR, NKC>(J, frags + sc.frag_off, threadIdx.x & 63);
}

// Persistent form over a batch of tiles: every wave pulls items (scale j of
// the launch, tile, row segment, wave column) from a counter.  Items are
// numbered scale-major, so a launch finishes its scales in order.
template <int NKR, int NKC>
__global__ __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(mfma_batch_waves<NKC>(), 2)))
void log_mfma_u8_batch_kernel(
    int n_tiles, const BatchTile* __restrict__ tiles, float* __restrict__ stack,
    const half8_t* __restrict__ frags, MfmaBatchScales sc, BatchCounters* __restrict__ ctr,
    int slot) {
    const int lane = threadIdx.x & 63;
    const int per_scale = ctr->mitems_per_scale;
    const int total = ctr->valid ? per_scale * sc.n : 0;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(&ctr->mwork[slot], 1);
        item = __shfl(item, 0, 64);
        if (item >= total) break;
        const int j = item / per_scale;
        const int rem = item - j * per_scale;
        int lo = 0, hi = n_tiles;  // last tile with mitem_base <= rem
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tiles[mid].mitem_base <= rem)
                lo = mid;
            else
                hi = mid;
        }
        const BatchTile& t = tiles[lo];
        const int local = rem - t.mitem_base;
        const int seg = local / t.mtiles_x;
        const int wcol = local - seg * t.mtiles_x;
        WaveJob J;
        J.img = static_cast<const uint8_t*>(t.img);
        J.pitch = t.pitch;
        J.h = t.h;
        J.w = t.w;
        J.plane = stack + t.stack_off + static_cast<long long>(sc.plane[j]) * t.h * t.w;
        J.x0 = wcol * 16 * WT;
        J.y0 = seg * t.mseg_rows;
        J.y1 = min(J.y0 + t.mseg_rows, t.h);
        J.rw8 = sc.rw8[j];
        J.rwc = sc.rwc[j];
        J.aligned = (t.pitch % 8 == 0) && (reinterpret_cast<uintptr_t>(t.img) % 8 == 0);
        J.out_vec = (t.w % 4 == 0) && (t.stack_off % 4 == 0) &&
                    (reinterpret_cast<uintptr_t>(stack) % 16 == 0);
        J.out_scale = sc.out_scale[j];
        run_job<NKR, NKC>(J, frags + sc.frag_off[j], lane);
    }
}

template <int NKR, int NKC>
hipError_t launch_one(const uint8_t* img, int h, int w, int64_t pitch, const uint16_t* frags,
                      const MfmaLaunch& L, float* out, long long plane_stride, hipStream_t s) {
    int blocks = 0;
    for (int i = 0; i < L.n; ++i) blocks += L.sc[i].n_blocks;
    if (blocks == 0) return hipSuccess;
    const int aligned = (pitch % 8 == 0) && (reinterpret_cast<uintptr_t>(img) % 8 == 0);
    // float4 stores need 16-byte aligned rows and planes
    const int out_vec = (w % 4 == 0) && (plane_stride % 4 == 0) &&
                        (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    log_mfma_u8_kernel<NKR, NKC><<<blocks, 64 * MW, 0, s>>>(
        img, h, w, static_cast<long long>(pitch), aligned, out_vec,
        reinterpret_cast<const half8_t*>(frags), L, out, plane_stride);
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

hipError_t launch_log_mfma_batch(int nkr, int nkc, int n_tiles, const BatchTile* tiles,
                                 float* stack, const uint16_t* frags, const MfmaBatchScales& sc,
                                 BatchCounters* ctr, int slot, int grid, hipStream_t s) {
    if (sc.n == 0) return hipSuccess;
    const half8_t* f = reinterpret_cast<const half8_t*>(frags);
#define MHFD_MFMA_BATCH_CASE(A, B)                                                        \
    if (nkr == A && nkc == B) {                                                           \
        log_mfma_u8_batch_kernel<A, B><<<grid, 64 * MW, 0, s>>>(n_tiles, tiles, stack, f, sc, \
                                                                ctr, slot);               \
        return hipGetLastError();                                                         \
    }
    MHFD_MFMA_BATCH_CASE(1, 1)
    MHFD_MFMA_BATCH_CASE(2, 2)
    MHFD_MFMA_BATCH_CASE(3, 3)
    MHFD_MFMA_BATCH_CASE(4, 4)
#undef MHFD_MFMA_BATCH_CASE
    return hipErrorInvalidValue;
}
int mfma_waves_per_block() { return MW; }

hipError_t launch_log_mfma(int nkr, int nkc, const uint8_t* img, int h, int w, int64_t pitch,
                           const uint16_t* frags, const MfmaLaunch& L, float* out,
                           long long plane_stride, hipStream_t s) {
#define MHFD_MFMA_CASE(A, B) \
    if (nkr == A && nkc == B) return launch_one<A, B>(img, h, w, pitch, frags, L, out, plane_stride, s);
    MHFD_MFMA_CASE(1, 1)
    MHFD_MFMA_CASE(2, 2)
    MHFD_MFMA_CASE(3, 3)
    MHFD_MFMA_CASE(4, 4)
#undef MHFD_MFMA_CASE
    return hipErrorInvalidValue;
}

}  // namespace mhfd
