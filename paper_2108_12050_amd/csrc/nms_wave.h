// 3x3x3 maxima, threshold and per-cell compaction for one wave: the body
// shared by the single-tile and the batched maxima kernels.
#pragma once

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "mhfd_internal.h"

namespace mhfd {
namespace nms {

constexpr int ROWS = 16;  // rows per wave

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
// run with row y+2 already in flight; the row loop is unrolled by the four
// row buffers, so rolling renames registers instead of moving them.
// Horizontal neighbours come from DPP wave shifts; the two columns beyond
// the strip (x0 - 1 and x0 + 64 CW) of every plane come from one more load
// per row (lanes k and 32 + k hold plane k's left and right halo), reduced
// vertically in those lanes and read out per plane.
//
// Borders replicate the edge row or column (reads are clamped into the
// image): a 3 x 3 maximum over a window that repeats one of its own members
// equals the maximum over the members inside the image, which is what the
// -inf padding of the definition gives.  Lanes past the right edge hold
// the last CW columns, report no candidates and pass column W - 1 on as
// the right neighbour of the last column inside.
//
// Every (row, strip) cell compacts its candidates in (x, k) order with
// ballot/mbcnt offsets into its own pool slot and reserves the overflow
// region with one atomic only when it has more.
//
// Threshold-sparse stacks (SPARSE, tau >= 0): the LoG wrote only the
// 4-pixel row groups holding a value above tau, and marked them in `act`
// (bit 16 g + r of word [k][by][bx]: row 16 by + r, columns 16 bx + 4 g
// ... + 3; every word is written).  A value at or below tau can neither be
// a candidate nor block one (a blocking neighbour exceeds the candidate,
// which exceeds tau), so any value at or below tau may stand in for it:
// unmarked groups, and rows outside the image, read as 0 <= tau.  The
// decisions are those of the dense stack, and only marked groups are
// fetched.
//
// Third word of a raw buffer resource on gfx9-family devices (32-bit data
// format, no swizzle): loads past its num_records return 0.
constexpr int kBufferFlags = 0x00020000;

struct Active {
    const uint64_t* mask;  // K x mby x mbx words
    int mbx, mby;
};

template <int K, int CW, int SLOTS, bool SPARSE = false>
__device__ __forceinline__ void wave(const float* __restrict__ st, int H, int W, float tau,
                                     int bpr, int strip, int run, const Sink& out,
                                     const Active& act = Active{nullptr, 0, 0}) {
    static_assert(CW * K <= 64, "candidate mask is 64 bits");
    // a lane's (column, plane) hits, bit c K + k
    typedef typename std::conditional<(CW * K > 32), unsigned long long, unsigned>::type Mask;
    typedef float Vec __attribute__((ext_vector_type(CW)));
    typedef Vec Row[K];
    const int lane = threadIdx.x & 63;
    const int x0 = strip * 64 * CW;
    const int xl = x0 + CW * lane;            // first column of the lane
    const bool col_ok = xl < W;               // W % CW == 0: all CW columns or none
    const int xc = col_ok ? xl : W - CW;
    const size_t plane = static_cast<size_t>(H) * W;
    const int y0 = run * ROWS;
    const int y1 = min(y0 + ROWS, H);
    // halo lane: plane hk, column hx (clamped into the image)
    const int hk = (lane & 31) < K ? (lane & 31) : 0;
    const int hx = min(max(lane < 32 ? x0 - 1 : x0 + 64 * CW, 0), W - 1);
    const float* __restrict__ hbase = st + static_cast<size_t>(hk) * plane + hx;

    // SPARSE: marks of rows y0 - 1 ... y0 + 16 (bit i: row y0 - 1 + i) of the
    // lane's group in every plane, and of the halo lane's group.
    uint32_t abits[SPARSE ? K : 1] = {};
    uint32_t hbits = 0;
    if constexpr (SPARSE) {
        const int by = y0 >> 4;
        // The three words are loaded unconditionally (rows clamped into the
        // image) so that their loads overlap; the selects drop the rows
        // outside it.
        auto run_bits = [&](int k, int x) -> uint32_t {
            const int sh = 16 * ((x >> 2) & 3);
            const uint64_t* m = act.mask + static_cast<size_t>(k) * act.mby * act.mbx + (x >> 4);
            const uint64_t wu = m[static_cast<size_t>(max(by - 1, 0)) * act.mbx];
            const uint64_t wc = m[static_cast<size_t>(by) * act.mbx];
            const uint64_t wd = m[static_cast<size_t>(min(by + 1, act.mby - 1)) * act.mbx];
            const uint32_t cur = static_cast<uint32_t>(wc >> sh) & 0xFFFFu;
            const uint32_t up = y0 > 0 ? static_cast<uint32_t>(wu >> (sh + 15)) & 1u : 0u;
            const uint32_t dn = y0 + 16 < H ? static_cast<uint32_t>(wd >> sh) & 1u : 0u;
            return up | (cur << 1) | (dn << 17);
        };
#pragma unroll
        for (int k = 0; k < K; ++k) abits[k] = run_bits(k, xc);
        hbits = run_bits(hk, hx);
    }

    // Plane k's rows start at the wave-uniform st + k plane; the lane's part
    // is a 32-bit byte offset (a plane holds fewer than 2^29 pixels).
    auto load_row = [&](int y, Row& v, float& hv) {
        const int yy = min(max(y, 0), H - 1);
        const uint32_t boff = static_cast<uint32_t>(yy * W + xc) * 4u;
        const int bit = y - y0 + 1;  // 0 .. 18
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const char* pk = reinterpret_cast<const char*>(st + static_cast<size_t>(k) * plane);
            if constexpr (SPARSE) {
                // Unmarked groups: an offset past the plane, for which the
                // buffer load fetches nothing and returns 0 (no branch).
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<char*>(pk), static_cast<short>(0),
                    static_cast<int>(static_cast<uint32_t>(plane * 4)), kBufferFlags);
                const uint32_t off = (abits[k] >> bit) & 1u ? boff : 0x80000000u;
                if constexpr (CW == 1)
                    v[k] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
                else if constexpr (CW == 2)
                    v[k] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                else
                    v[k] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
            } else {
                v[k] = *reinterpret_cast<const Vec*>(pk + boff);
            }
        }
        if constexpr (SPARSE)
            hv = (hbits >> bit) & 1u ? hbase[static_cast<size_t>(yy) * W] : 0.0f;
        else
            hv = hbase[static_cast<size_t>(yy) * W];
    };
    auto test_row = [&](int y, const Row& up, const Row& cur, const Row& dn, float hup,
                        float hcur, float hdn) {
        const float hm = fmax3(hup, hcur, hdn);
        // 3x3 maxima of plane k (vertical, then horizontal with DPP shifts
        // and the halo lanes at the strip ends)
        auto plane_max = [&](int k) {
            Vec vm, m;
#pragma unroll
            for (int c = 0; c < CW; ++c) vm[c] = fmax3(up[k][c], cur[k][c], dn[k][c]);
            // a lane past the right edge holds columns W - CW .. W - 1 and
            // hands column W - 1 to the last lane inside (the replicated edge)
            const float left = wave_shr1(vm[CW - 1], lane_value(hm, k));
            const float right = wave_shl1(col_ok ? vm[0] : vm[CW - 1], lane_value(hm, 32 + k));
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const float l = c > 0 ? vm[c - 1] : left;
                const float r = c + 1 < CW ? vm[c + 1] : right;
                m[c] = fmax3(l, vm[c], r);
            }
            return m;
        };
        // planes k - 1, k, k + 1 in a rolling window
        Mask mask = 0u;
        Vec mp = static_cast<Vec>(-INFINITY), mk = plane_max(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const Vec mn = k + 1 < K ? plane_max(k + 1) : static_cast<Vec>(-INFINITY);
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const float v = cur[k][c];
                const bool hit = (v > tau) & (v >= fmax3(mp[c], mk[c], mn[c]));
                mask |= static_cast<Mask>(hit) << (c * K + k);
            }
            mp = mk;
            mk = mn;
        }
        mask = col_ok ? mask : Mask(0);
        const int64_t cell = static_cast<int64_t>(y) * bpr + strip;
        if (__ballot(mask != 0u) == 0ull) {  // wave-uniform: no candidate in the cell
            if (lane == 0) {
                out.blk_n[cell] = 0;
                out.blk_o[cell] = 0;
            }
            return;
        }
        const int cnt = static_cast<int>(__popcll(static_cast<unsigned long long>(mask)));
        int n;
        const int pre = wave_exclusive_prefix<6>(cnt, &n);
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
        // The lane's candidates in (x, k) order: set bits of the mask from
        // the lowest; the response is read back from the stack (cached).
        if (cnt > 0) {
            int j = pre;
            Cand* own = out.slots + cell * SLOTS;
            Mask m = mask;
            do {
                const int bit = __builtin_ctzll(static_cast<unsigned long long>(m));
                m &= m - 1;
                const int c = bit / K;
                const int k = bit - c * K;
                Cand rec;
                rec.y = y;
                rec.x = xl + c;
                rec.k = k | out.k_tag;
                rec.r = st[static_cast<size_t>(k) * plane + static_cast<size_t>(y) * W + xl + c];
                if (j < SLOTS)
                    own[j] = rec;
                else if (o + (j - SLOTS) < out.cap)
                    out.over[o + (j - SLOTS)] = rec;
                ++j;
            } while (m);
        }
    };
    Row b0, b1, b2, b3;
    float h0, h1, h2, h3;
    load_row(y0 - 1, b0, h0);
    load_row(y0, b1, h1);
    load_row(y0 + 1, b2, h2);
    // rows y-1, y, y+1 in (b0, b1, b2) at the top of every pass
    for (int y = y0; y < y1; y += 4) {
        load_row(y + 2, b3, h3);
        test_row(y, b0, b1, b2, h0, h1, h2);
        if (y + 1 >= y1) break;
        load_row(y + 3, b0, h0);
        test_row(y + 1, b1, b2, b3, h1, h2, h3);
        if (y + 2 >= y1) break;
        load_row(y + 4, b1, h1);
        test_row(y + 2, b2, b3, b0, h2, h3, h0);
        if (y + 3 >= y1) break;
        load_row(y + 5, b2, h2);
        test_row(y + 3, b3, b0, b1, h3, h0, h1);
    }
}

}  // namespace nms
}  // namespace mhfd
