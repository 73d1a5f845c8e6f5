// 3x3x3 maxima, threshold and per-cell compaction for one wave: the body
// shared by the single-tile and the batched maxima kernels.
#pragma once

#include <math.h>
#include <stdint.h>

#include "mhfd_internal.h"

namespace mhfd {
namespace nms {

constexpr int ROWS = 32;  // rows per wave

__device__ __forceinline__ float fmax3(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }

// Exclusive prefix within the wave of a per-lane count c in [0, 2^bits).
template <int BITS>
__device__ __forceinline__ int wave_exclusive_prefix(int c, int* wave_total) {
    int pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const unsigned long long bal = __ballot((c >> b) & 1);
        const unsigned lo = static_cast<unsigned>(bal);
        const unsigned hi = static_cast<unsigned>(bal >> 32);
        pre += static_cast<int>(__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u))) << b;
        tot += __popcll(bal) << b;
    }
    *wave_total = tot;
    return pre;
}

// Neighbour exchange across the whole wave (DPP wave shifts, no LDS): lane l
// receives lane l - 1's value (shr) or lane l + 1's (shl); the lane without
// a source receives `edge`.
__device__ __forceinline__ float wave_shr1(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, edge), __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ float wave_shl1(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, edge), __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}

// Where one wave's candidates go: the cells of its tile (counts, overflow
// offsets, SLOTS-record pool slots), the shared overflow region and its
// counters, and a tag OR-ed into every record's k.
struct Sink {
    int32_t* blk_n;     // tile's first cell
    int32_t* blk_o;
    Cand* slots;        // tile's first cell's slot
    Cand* over;         // shared overflow region
    int64_t cap;        // overflow records
    int32_t* pool_used;
    int32_t* flags;
    int k_tag;
};

// One wave over strip `strip` (64 CW columns) and rows [ROWS run, ...) of a
// K x H x W stack.  Lane l owns columns x0 + CW l ... x0 + CW l + CW - 1,
// read as one aligned CW-float load per plane and row (W % CW == 0).  The
// wave keeps rows y-1, y, y+1 of every plane in registers, rolling down the
// run with row y+2 already in flight.  Horizontal neighbours come from DPP
// wave shifts; the two columns beyond the strip (x0 - 1 and x0 + 64 CW) of
// every plane come from one more load per row (lanes k and 32 + k hold plane
// k's left and right halo), reduced vertically in those lanes and read out
// per plane.  Every (row, strip) cell compacts its candidates in (x, k)
// order with ballot/mbcnt offsets into its own pool slot and reserves the
// overflow region with one atomic only when it has more.
template <int K, int CW, int SLOTS>
__device__ __forceinline__ void wave(const float* __restrict__ st, int H, int W, float tau,
                                     int bpr, int strip, int run, const Sink& out) {
    static_assert(CW * K <= 32, "candidate mask is 32 bits");
    typedef float Vec __attribute__((ext_vector_type(CW)));
    const int lane = threadIdx.x & 63;
    const int x0 = strip * 64 * CW;
    const int xl = x0 + CW * lane;            // first column of the lane
    const bool col_ok = xl < W;               // W % CW == 0: all CW columns or none
    const int xc = col_ok ? xl : W - CW;
    const size_t plane = static_cast<size_t>(H) * W;
    const int y0 = run * ROWS;
    const int y1 = min(y0 + ROWS, H);
    // halo lane: plane hk, column hx
    const int hk = lane & 31;
    const int hx = lane < 32 ? x0 - 1 : x0 + 64 * CW;
    const bool h_ok = hk < K && hx >= 0 && hx < W;
    const size_t h_off = static_cast<size_t>(h_ok ? hk : 0) * plane + (h_ok ? hx : 0);

    auto load_row = [&](int y, Vec* v, float& hv) {
        const bool ok = y >= 0 && y < H;
        const int yy = y < 0 ? 0 : (y >= H ? H - 1 : y);
        const float* p = st + static_cast<size_t>(yy) * W + xc;
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = *reinterpret_cast<const Vec*>(p + k * plane);
        hv = st[h_off + static_cast<size_t>(yy) * W];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (ok && col_ok) ? v[k] : static_cast<Vec>(-INFINITY);
        hv = (ok && h_ok) ? hv : -INFINITY;
    };
    Vec up[K], cur[K], dn[K], nx[K];
    float hup, hcur, hdn, hnx;
    load_row(y0 - 1, up, hup);
    load_row(y0, cur, hcur);
    load_row(y0 + 1, dn, hdn);
    for (int y = y0; y < y1; ++y) {
        load_row(y + 2, nx, hnx);  // in flight while row y is tested
        const float hm = fmax3(hup, hcur, hdn);
        Vec m3[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Vec vm;
#pragma unroll
            for (int c = 0; c < CW; ++c) vm[c] = fmax3(up[k][c], cur[k][c], dn[k][c]);
            const float left = wave_shr1(vm[CW - 1], lane_value(hm, k));
            const float right = wave_shl1(vm[0], lane_value(hm, 32 + k));
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const float l = c > 0 ? vm[c - 1] : left;
                const float r = c + 1 < CW ? vm[c + 1] : right;
                m3[k][c] = fmax3(l, vm[c], r);
            }
        }
        unsigned mask = 0u;
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float mp = k > 0 ? m3[k - 1][c] : -INFINITY;
                const float mn = k + 1 < K ? m3[k + 1][c] : -INFINITY;
                const float v = cur[k][c];
                if (v > tau && v >= fmax3(mp, m3[k][c], mn)) mask |= 1u << (c * K + k);
            }
        const int cnt = __popc(mask);
        int n;
        const int pre = wave_exclusive_prefix<6>(cnt, &n);
        const int64_t cell = static_cast<int64_t>(y) * bpr + strip;
        int o = 0;
        if (lane == 0) {
            if (n > SLOTS) {
                o = atomicAdd(out.pool_used, n - SLOTS);
                if (static_cast<int64_t>(o) + (n - SLOTS) > out.cap)
                    atomicOr(out.flags, MHFD_FLAG_CAND_OVERFLOW);
            }
            out.blk_n[cell] = n;
            out.blk_o[cell] = o;
        }
        o = __shfl(o, 0, 64);
        if (cnt > 0) {
            int j = pre;
            Cand* own = out.slots + cell * SLOTS;
            Cand* over = out.over + o - SLOTS;
#pragma unroll
            for (int c = 0; c < CW; ++c)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (mask & (1u << (c * K + k))) {
                        Cand rec;
                        rec.y = y;
                        rec.x = xl + c;
                        rec.k = k | out.k_tag;
                        rec.r = cur[k][c];
                        if (j < SLOTS)
                            own[j] = rec;
                        else if (o + (j - SLOTS) < out.cap)
                            over[j] = rec;
                        ++j;
                    }
                }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            up[k] = cur[k];
            cur[k] = dn[k];
            dn[k] = nx[k];
        }
        hup = hcur;
        hcur = hdn;
        hdn = hnx;
    }
}

}  // namespace nms
}  // namespace mhfd
