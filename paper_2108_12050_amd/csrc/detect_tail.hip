// Detection after the LoG stack: 3x3x3 maxima, threshold, compaction into
// canonical (y, x, k) order, one-shot overlap pruning, blob list.
//
//   nms        one wave per (strip of 64 CW columns, run of 16 rows); a lane
//              owns CW adjacent columns and walks down the rows, taking its
//              neighbours' edge columns by DPP shifts.  A voxel is a candidate when
//              it equals the maximum of its 3x3x3 window (the maxpool-equality
//              test of section 3, taken local in scale too) and is above the
//              threshold.  Counts per lane become in-wave offsets with ballot
//              + mbcnt over the bits of the count; every (row, strip) cell
//              owns a pool slot.
//   scan       exclusive scan of the per-cell counts in cell order, i.e. in
//              (y, x) order: the canonical position of every cell's run.
//   order      copies each run from the pool to its canonical place.
//   prune      one work item per (candidate, row offset) searches that row
//              (row ranges come from the scan) for a dominating candidate
//              within the plan's integer overlap distance, the exact form of
//              the FP64 lens-overlap test.
//   emit       scan of the keep flags, then the blob records.
// No step depends on the order in which workgroups run, so the output is
// deterministic.
#include <float.h>
#include <math.h>

#include <utility>

#include "mhfd_internal.h"
#include "nms_wave.h"

namespace mhfd {

namespace {

constexpr int NMS_WAVES = 4;   // independent waves per NMS workgroup
constexpr int SLOT = 16;       // pool records each (row, strip) cell owns
constexpr int SCAN_T = 1024;

using nms::fmax3;
using nms::wave_exclusive_prefix;

__global__ void init_counters_kernel(DetectCounters* ctr) {
    if (threadIdx.x == 0) {
        ctr->pool_used = 0;
        ctr->flags = 0;
        ctr->n_cand = 0;
        ctr->n_blobs = 0;
    }
}

// One wave per (strip of 64 CW columns, run of nms::ROWS rows); a workgroup
// holds NMS_WAVES independent waves.  The per-wave body is nms::wave.
template <int K, int CW, bool SPARSE>
__global__ __launch_bounds__(64 * NMS_WAVES) void nms_kernel(
    const float* __restrict__ st, int H, int W, float tau, int bpr, int n_runs,
    int32_t* __restrict__ blk_n, int32_t* __restrict__ blk_o, Cand* __restrict__ pool,
    int64_t n_cells, int64_t cap, DetectCounters* __restrict__ ctr, nms::Active act) {
    // (run, strip), strip fastest; wave-uniform (readfirstlane), so the row
    // and column bookkeeping stays in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * NMS_WAVES + (threadIdx.x >> 6));
    if (wid >= n_runs * bpr) return;
    nms::Sink out;
    out.blk_n = blk_n;
    out.blk_o = blk_o;
    out.slots = pool;
    out.over = pool + n_cells * SLOT;
    out.cap = cap;
    out.pool_used = &ctr->pool_used;
    out.flags = &ctr->flags;
    out.k_tag = 0;
    nms::wave<K, CW, SLOT, SPARSE>(st, H, W, tau, bpr, wid % bpr, wid / bpr, out, act);
}

template <int K, int CW>
void launch_nms_k(const DetectWorkspace& ws, int h, int w, float tau, hipStream_t s) {
    const int runs = (h + nms::ROWS - 1) / nms::ROWS;
    const int waves = runs * ws.blk_per_row;
    const int grid = (waves + NMS_WAVES - 1) / NMS_WAVES;
    const nms::Active act{ws.act, ws.act_bx, ws.act_by};
    if (ws.act)
        nms_kernel<K, CW, true><<<grid, 64 * NMS_WAVES, 0, s>>>(
            ws.stack, h, w, tau, ws.blk_per_row, runs, ws.blk_n, ws.blk_o, ws.pool, ws.n_blk,
            ws.cap, ws.ctr, act);
    else
        nms_kernel<K, CW, false><<<grid, 64 * NMS_WAVES, 0, s>>>(
            ws.stack, h, w, tau, ws.blk_per_row, runs, ws.blk_n, ws.blk_o, ws.pool, ws.n_blk,
            ws.cap, ws.ctr, act);
}

template <int... Ks>
void launch_nms(int K, int cw, const DetectWorkspace& ws, int h, int w, float tau, hipStream_t s,
                std::integer_sequence<int, Ks...>) {
    if (cw == 4) {
        ((K == Ks + 1 && Ks + 1 <= 10 ? launch_nms_k<Ks + 1, (Ks + 1 <= 10 ? 4 : 1)>(ws, h, w, tau, s)
                                     : void()), ...);
    } else if (cw == 2) {
        ((K == Ks + 1 && Ks + 1 <= 16 ? launch_nms_k<Ks + 1, (Ks + 1 <= 16 ? 2 : 1)>(ws, h, w, tau, s)
                                      : void()), ...);
    } else {
        ((K == Ks + 1 ? launch_nms_k<Ks + 1, 1>(ws, h, w, tau, s) : void()), ...);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan over n = min(n_host, *n_dev) ints in three launches:
// per-span sums, a scan of the span sums by one workgroup, per-span scans.
constexpr int SCAN_BT = 256;              // threads per span workgroup
constexpr int SCAN_ITEMS = 16;            // items per thread
constexpr int SCAN_SPAN = SCAN_BT * SCAN_ITEMS;

__device__ __forceinline__ int scan_n(int n_host, const int32_t* n_dev) {
    return n_dev ? min(n_host, *n_dev) : n_host;
}

// Inclusive scan of one int per thread across a workgroup of SCAN_BT threads.
__device__ __forceinline__ int block_inclusive_scan(int v, int* sh /* SCAN_BT/64 ints */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    if (lane == 63) sh[wv] = v;
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int i = 0; i < SCAN_BT / 64; ++i) add += i < wv ? sh[i] : 0;
    return v + add;
}

__global__ __launch_bounds__(SCAN_BT) void scan_sums_kernel(const int32_t* __restrict__ in,
                                                           int n_host,
                                                           const int32_t* __restrict__ n_dev,
                                                           int32_t* __restrict__ sums) {
    __shared__ int sh[SCAN_BT / 64];
    const int n = scan_n(n_host, n_dev);
    const int base = blockIdx.x * SCAN_SPAN + threadIdx.x * SCAN_ITEMS;
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    const int incl = block_inclusive_scan(s, sh);
    if (threadIdx.x == SCAN_BT - 1) sums[blockIdx.x] = incl;
}

// Exclusive scan of the nb span sums in place; writes the total to out[n]
// and to *total_out if given.
__global__ __launch_bounds__(1024) void scan_top_kernel(int32_t* __restrict__ sums, int nb,
                                                        int n_host,
                                                        const int32_t* __restrict__ n_dev,
                                                        int32_t* __restrict__ out,
                                                        int32_t* __restrict__ total_out) {
    __shared__ int sh[1024];
    const int n = scan_n(n_host, n_dev);
    const int nb_used = (n + SCAN_SPAN - 1) / SCAN_SPAN;
    int carry = 0;
    for (int b0 = 0; b0 < nb_used; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb_used ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int t = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb_used) sums[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    (void)nb;
    if (threadIdx.x == 0) {
        out[n] = carry;
        if (total_out) *total_out = carry;
    }
}

__global__ __launch_bounds__(SCAN_BT) void scan_apply_kernel(const int32_t* __restrict__ in,
                                                            int n_host,
                                                            const int32_t* __restrict__ n_dev,
                                                            const int32_t* __restrict__ sums,
                                                            int32_t* __restrict__ out) {
    __shared__ int sh[SCAN_BT / 64];
    const int n = scan_n(n_host, n_dev);
    if (blockIdx.x * SCAN_SPAN >= n) return;
    const int base = blockIdx.x * SCAN_SPAN + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int run = block_inclusive_scan(s, sh) - s + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// Second pass when there are at most SCAN_BT spans: every workgroup adds up
// the span sums before its own (one per thread) instead of a separate scan
// of the span sums, and the workgroup holding the last element writes the
// total.  Same result as scan_top_kernel + scan_apply_kernel, one launch.
__global__ __launch_bounds__(SCAN_BT) void scan_apply_small_kernel(
    const int32_t* __restrict__ in, int n_host, const int32_t* __restrict__ n_dev,
    const int32_t* __restrict__ sums, int32_t* __restrict__ out, int32_t* __restrict__ total_out) {
    __shared__ int sh[SCAN_BT / 64];
    __shared__ int offset;
    const int n = scan_n(n_host, n_dev);
    if (n == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            out[0] = 0;
            if (total_out) *total_out = 0;
        }
        return;
    }
    if (blockIdx.x * SCAN_SPAN >= n) return;  // whole workgroup
    {
        const int before = block_inclusive_scan(
            static_cast<int>(threadIdx.x) < static_cast<int>(blockIdx.x) ? sums[threadIdx.x] : 0, sh);
        if (threadIdx.x == SCAN_BT - 1) offset = before;
        __syncthreads();
    }
    const int base = blockIdx.x * SCAN_SPAN + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    const int incl = block_inclusive_scan(s, sh);
    int run = incl - s + offset;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == SCAN_BT - 1 && (n - 1) / SCAN_SPAN == static_cast<int>(blockIdx.x)) {
        out[n] = offset + incl;
        if (total_out) *total_out = offset + incl;
    }
}

void launch_scan(const int32_t* in, int n_host, const int32_t* n_dev, int32_t* sums,
                 int32_t* out, int32_t* total_out, hipStream_t s) {
    const int nb = (n_host + SCAN_SPAN - 1) / SCAN_SPAN;
    const int grid = nb > 0 ? nb : 1;
    scan_sums_kernel<<<grid, SCAN_BT, 0, s>>>(in, n_host, n_dev, sums);
    if (grid <= SCAN_BT) {
        scan_apply_small_kernel<<<grid, SCAN_BT, 0, s>>>(in, n_host, n_dev, sums, out, total_out);
        return;
    }
    scan_top_kernel<<<1, 1024, 0, s>>>(sums, grid, n_host, n_dev, out, total_out);
    scan_apply_kernel<<<grid, SCAN_BT, 0, s>>>(in, n_host, n_dev, sums, out);
}

// Also sets every candidate's keep flag to 1 (the prune clears flags).
__global__ void order_kernel(const int32_t* __restrict__ blk_off, const int32_t* __restrict__ blk_o,
                             int n_blk, const Cand* __restrict__ pool, Cand* __restrict__ cand,
                             int32_t* __restrict__ keep, int64_t cap,
                             const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    if (blockIdx.x == 0 && threadIdx.x == 0 && ctr->n_cand > cap)
        atomicOr(const_cast<int32_t*>(&ctr->flags), MHFD_FLAG_CAND_OVERFLOW);
    const Cand* over = pool + static_cast<int64_t>(n_blk) * SLOT;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        // last workgroup b with blk_off[b] <= i
        int lo = 0, hi = n_blk;  // invariant: blk_off[lo] <= i < blk_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (blk_off[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        const int j = static_cast<int>(i - blk_off[lo]);
        if (j < SLOT) {
            cand[i] = pool[static_cast<int64_t>(lo) * SLOT + j];
        } else {
            const int64_t src = static_cast<int64_t>(blk_o[lo]) + (j - SLOT);
            if (src < cap) cand[i] = over[src];
        }
        keep[i] = 1;
    }
}

// Overlap prune.  Candidates a that can remove b lie within `reach` rows
// and, in row y_b + dy, within |dx| <= sqrt(d2top - dy^2), d2top being the
// largest entry of the table (reach^2 can fall short of it); rows come from
// the per-row offsets of the canonical list and the column range from a
// binary search in the row (sorted by x).  The overlap test is the plan's
// exact integer form: overlap(a, b) > theta iff dy^2 + dx^2 <=
// d2max[k_a][k_b] (the lens fraction falls monotonically with distance; the
// table is evaluated in double on the host).
//
// One work item per (candidate, row offset): grid row blockIdx.y = dy +
// reach, and the workgroups of that row stride over the candidates.  keep[]
// starts at 1 (order_kernel); an item clears its candidate's flag when it
// finds a dominating candidate within the overlap distance in row y + dy.
// All writers write 0, so the order of the writes does not matter and the
// flags equal those of a scan over all rows.  Threads of a wave take
// consecutive candidates, which lie in nearly the same rows, so their
// searches share cache lines.
__global__ void prune_rows_kernel(const Cand* __restrict__ cand,
                                  const int32_t* __restrict__ blk_off, int bpr, int H, int K,
                                  const int32_t* __restrict__ d2max, int reach, int d2top,
                                  int32_t* __restrict__ keep, int64_t cap,
                                  const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    const long long dy = static_cast<long long>(blockIdx.y) - reach;
    const int xr = static_cast<int>(sqrt(static_cast<double>(d2top - dy * dy)));
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Cand b = cand[i];
        const long long yy = b.y + dy;
        if (yy < 0 || yy >= H || !keep[i]) continue;
        const int32_t* dcol = d2max + b.k;  // d2max[ka * K + kb]
        int lo = blk_off[yy * bpr];
        const int hi = min(static_cast<int64_t>(blk_off[(yy + 1) * bpr]), n);
        // first candidate of the row with x >= b.x - xr
        int top = hi;
        while (lo < top) {
            const int mid = (lo + top) >> 1;
            if (cand[mid].x < b.x - xr)
                lo = mid + 1;
            else
                top = mid;
        }
        for (int j = lo; j < hi; ++j) {
            const Cand a = cand[j];
            if (a.x > b.x + xr) break;
            const bool dom = a.k > b.k || (a.k == b.k && (a.y < b.y || (a.y == b.y && a.x < b.x)));
            const long long dx = a.x - b.x;
            if (dom && dy * dy + dx * dx <= dcol[a.k * K]) {
                keep[i] = 0;
                break;
            }
        }
    }
}

__global__ void emit_kernel(const Cand* __restrict__ cand, const int32_t* __restrict__ keep,
                            const int32_t* __restrict__ keep_off, const float* __restrict__ sigmas,
                            mhfd_blob* __restrict__ blobs, int capacity, int64_t cap,
                            double pixels, DetectCounters* __restrict__ ctr,
                            mhfd_result* __restrict__ result) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (!keep[i]) continue;
        const int32_t pos = keep_off[i];
        if (pos < capacity) {
            const Cand c = cand[i];
            mhfd_blob b;
            b.y = c.y;
            b.x = c.x;
            b.k = c.k;
            b.sigma = sigmas[c.k];
            b.response = c.r;
            blobs[pos] = b;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t nb = ctr->n_blobs;
        int32_t flags = ctr->flags;
        if (nb > capacity) flags |= MHFD_FLAG_BLOB_OVERFLOW;
        result->n_blobs = nb;
        result->n_candidates = ctr->n_cand;
        result->flags = flags;
        result->reserved = 0;
        result->density = static_cast<double>(nb) * 1e6 / pixels;
    }
}

}  // namespace

int nms_blocks_per_row(int w) { return (w + 63) / 64; }  // one column per lane: the most cells

void launch_batch_scan(const int32_t* in, int n_host, const int32_t* n_dev, int32_t* sums,
                       int32_t* out, int32_t* total_out, hipStream_t s) {
    launch_scan(in, n_host, n_dev, sums, out, total_out, s);
}

size_t nms_pool_records(int n_blk, int64_t cap) { return static_cast<size_t>(n_blk) * SLOT + cap; }

size_t scan_sums_ints(int64_t n) { return static_cast<size_t>((n + SCAN_SPAN - 1) / SCAN_SPAN + 1); }

hipError_t launch_detect_tail(const DetectWorkspace& ws, int K, int h, int w, float tau,
                              const int32_t* d2max, int reach, int d2top,
                              const float* sigmas_dev, mhfd_blob* blobs, int capacity,
                              mhfd_result* result, hipStream_t s) {
    init_counters_kernel<<<1, 64, 0, s>>>(ws.ctr);
    // Four columns per lane (float4 loads) for up to ten planes: per voxel
    // the strip-end exchange and the row bookkeeping cost half of what they
    // cost at two columns, and a wave keeps twice the bytes in flight
    // (K = 10: 219 registers, two waves per SIMD, 9% faster than two columns
    // at four waves; K = 1: 44 -> 36 us); two (float2) for 11 to 16 planes,
    // where four columns take 247 to 340 registers per lane (not measured).
    DetectWorkspace wk = ws;
    const uintptr_t sa = reinterpret_cast<uintptr_t>(ws.stack);
    const int cw = (K <= 10 && w % 4 == 0 && sa % 16 == 0) ? 4
                   : (K <= 16 && w % 2 == 0 && sa % 8 == 0) ? 2 : 1;
    wk.blk_per_row = (w + 64 * cw - 1) / (64 * cw);
    wk.n_blk = h * wk.blk_per_row;
    launch_nms(K, cw, wk, h, w, tau, s, std::make_integer_sequence<int, MHFD_MAX_SCALES>{});
    launch_scan(wk.blk_n, wk.n_blk, nullptr, ws.scan_sums, ws.blk_off, &ws.ctr->n_cand, s);
    const int grid = 1024;
    order_kernel<<<grid, 256, 0, s>>>(wk.blk_off, wk.blk_o, wk.n_blk, ws.pool, ws.cand, ws.keep,
                                      ws.cap, ws.ctr);
    if (d2max) {
        const int span = 2 * reach + 1;
        prune_rows_kernel<<<dim3(prune_grid_x(span), span), 256, 0, s>>>(
            wk.cand, wk.blk_off, wk.blk_per_row, h, K, d2max, reach, d2top, ws.keep, ws.cap,
            ws.ctr);
    }
    launch_scan(ws.keep, static_cast<int>(ws.cap), &ws.ctr->n_cand, ws.scan_sums, ws.keep_off,
                &ws.ctr->n_blobs, s);
    emit_kernel<<<grid, 256, 0, s>>>(ws.cand, ws.keep, ws.keep_off, sigmas_dev, blobs, capacity,
                                     ws.cap, static_cast<double>(h) * w, ws.ctr, result);
    return hipGetLastError();
}

}  // namespace mhfd
