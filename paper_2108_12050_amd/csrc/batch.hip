// Batched detection of tiles of different sizes from one fixed launch
// sequence.  The host never reads the tile descriptors: the setup kernel
// checks them and builds the per-tile table, so the sequence can be captured
// in a HIP graph and replayed with new descriptors.
//
//   setup      validate, per-tile LoG items / maxima cells and items / stack offsets
//              and their prefix sums (one workgroup);
//   LoG        persistent matrix-core waves per K-block shape (log_mfma.hip;
//              fp32 plans after a per-tile max |I| pass), the same per-wave
//              arithmetic as the single-tile path; scales above the
//              matrix-core radius: persistent strip workgroups per radius
//              class (log_strip.hip);
//   nms        persistent waves over every tile's (16-row run, strip) items,
//              the per-wave body of the single-tile path (nms_wave.h); the
//              tile index rides in the upper bits of k;
//   scan       over all cells, tile-major: the canonical list of every tile
//              is one contiguous run of the global list;
//   order, prune (rows of the candidate's own tile), keep scan, emit into the
//              tile's buffer, per-tile results.
#include <math.h>

#include <utility>

#include "mhfd_internal.h"
#include "nms_wave.h"

namespace mhfd {

namespace {

constexpr int NMS_WAVES = 4;   // maxima waves per workgroup
constexpr int SLOT = 16;
constexpr int SETUP_T = 1024;
constexpr int TILE_SHIFT = 5;  // k in the low bits (K <= 32), tile above

__device__ int default_seg_rows(int h, int w) {
    const int strips = (w + 63) / 64;
    long long seg = (static_cast<long long>(h) * strips + 1023) / 1024;
    seg = (seg + 31) / 32 * 32;
    if (seg < 32) seg = 32;
    if (seg > 1024) seg = 1024;
    return static_cast<int>(seg);
}

// Exclusive block scan of per-thread values (SETUP_T threads).
template <typename V>
__device__ V block_exclusive_scan(V v, V* sh, V* total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < SETUP_T; d <<= 1) {
        const V t = threadIdx.x >= d ? sh[threadIdx.x - d] : V(0);
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const V incl = sh[threadIdx.x];
    *total = sh[SETUP_T - 1];
    __syncthreads();
    return incl - v;
}

__device__ __forceinline__ int nms_runs(int h) { return (h + nms::ROWS - 1) / nms::ROWS; }

// Floats of a tile's K planes in the stack, rounded up to whole float4s so
// every tile starts 16-byte aligned.
__device__ __forceinline__ long long stack_floats(int h, int w, int K) {
    return (static_cast<long long>(h) * w * K + 3) / 4 * 4;
}

// Activity words of a tile's threshold-sparse stack.
__device__ __forceinline__ long long act_words(int h, int w, int K) {
    return static_cast<long long>(K) * ((h + 15) / 16) * ((w + 15) / 16);
}

// Rows per matrix-core work item: a wave recomputes 2 nkc - 1 intermediate
// blocks of 16 rows per item, so items are tall unless the tile is short.
__device__ int default_mfma_seg_rows(int h) {
    const int hr = (h + 15) / 16 * 16;
    return hr < 1024 ? hr : 1024;
}

__global__ __launch_bounds__(SETUP_T) void batch_setup_kernel(
    const mhfd_tile* __restrict__ in, int n, long long max_pixels, int K, int max_h, int max_w,
    int dtype, int mfma, BatchTile* __restrict__ tiles, BatchCounters* __restrict__ ctr) {
    __shared__ long long shl[SETUP_T];
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    const int per = (n + SETUP_T - 1) / SETUP_T;
    const int t0 = min(n, static_cast<int>(threadIdx.x) * per), t1 = min(n, t0 + per);
    long long items = 0, nms = 0, pix = 0, mitems = 0, nitems = 0, sfl = 0, acw = 0;
    for (int t = t0; t < t1; ++t) {
        const mhfd_tile d = in[t];
        bool ok = d.img && d.result && d.h >= 1 && d.w >= 1 && d.h <= max_h && d.w <= max_w &&
                  d.pitch >= d.w && d.capacity >= 0 && (d.capacity == 0 || d.blobs) &&
                  (d.seg_rows == 0 || (d.seg_rows % 32 == 0 && d.seg_rows >= 32 && d.seg_rows <= 4096)) &&
                  (dtype == MHFD_U8 || (reinterpret_cast<uintptr_t>(d.img) & 3) == 0);
        if (!ok) atomicOr(&bad_s, 1);
        BatchTile bt{};
        bt.img = d.img;
        bt.pitch = d.pitch;
        bt.blobs = d.blobs;
        bt.result = d.result;
        bt.h = ok ? d.h : 1;
        bt.w = ok ? d.w : 1;
        bt.capacity = ok ? d.capacity : 0;
        bt.seg_rows = ok ? (d.seg_rows ? d.seg_rows : default_seg_rows(d.h, d.w)) : 32;
        bt.strips = (bt.w + 63) / 64;
        bt.segs = (bt.h + bt.seg_rows - 1) / bt.seg_rows;
        // four columns per maxima lane up to ten planes when every row of the
        // tile starts 16-byte aligned (tiles start on whole float4s, so
        // w % 4 == 0 suffices), two up to 16 planes on even widths (as the
        // single-tile pass chooses)
        bt.nms_cw = (K <= 10 && bt.w % 4 == 0) ? 4 : (K <= 16 && bt.w % 2 == 0) ? 2 : 1;
        bt.bpr = (bt.w + 64 * bt.nms_cw - 1) / (64 * bt.nms_cw);
        bt.mseg_rows = d.seg_rows && ok ? d.seg_rows : default_mfma_seg_rows(bt.h);
        bt.mtiles_x = mfma ? (bt.w + MFMA_WAVE_COLS - 1) / MFMA_WAVE_COLS : 0;
        bt.mgroups_x = (bt.mtiles_x + MFMA_GROUP_WAVES - 1) / MFMA_GROUP_WAVES;
        bt.msegs = (bt.h + bt.mseg_rows - 1) / bt.mseg_rows;
        tiles[t] = bt;
        mitems += static_cast<long long>(bt.mgroups_x) * bt.msegs;
        items += static_cast<long long>(bt.strips) * bt.segs;
        nms += static_cast<long long>(bt.h) * bt.bpr;
        nitems += static_cast<long long>(nms_runs(bt.h)) * bt.bpr;
        pix += static_cast<long long>(bt.h) * bt.w;
        sfl += stack_floats(bt.h, bt.w, K);
        acw += act_words(bt.h, bt.w, K);
    }
    long long tot_items, tot_nms, tot_pix, tot_mitems, tot_nitems, tot_sfl;
    const long long b_items = block_exclusive_scan(items, shl, &tot_items);
    const long long b_nms = block_exclusive_scan(nms, shl, &tot_nms);
    const long long b_pix = block_exclusive_scan(pix, shl, &tot_pix);
    const long long b_mitems = block_exclusive_scan(mitems, shl, &tot_mitems);
    const long long b_nitems = block_exclusive_scan(nitems, shl, &tot_nitems);
    const long long b_sfl = block_exclusive_scan(sfl, shl, &tot_sfl);
    long long tot_acw;
    const long long b_acw = block_exclusive_scan(acw, shl, &tot_acw);
    (void)b_pix;
    (void)tot_sfl;
    (void)tot_acw;
    long long ri = b_items, rn = b_nms, rm = b_mitems, rq = b_nitems, rs = b_sfl, ra = b_acw;
    for (int t = t0; t < t1; ++t) {
        BatchTile& bt = tiles[t];
        bt.item_base = static_cast<int>(ri);
        bt.nms_base = static_cast<int>(rn);
        bt.mitem_base = static_cast<int>(rm);
        bt.nitem_base = static_cast<int>(rq);
        bt.stack_off = rs;
        bt.act_off = ra;
        ra += act_words(bt.h, bt.w, K);
        ri += static_cast<long long>(bt.strips) * bt.segs;
        rn += static_cast<long long>(bt.h) * bt.bpr;
        rm += static_cast<long long>(bt.mgroups_x) * bt.msegs;
        rq += static_cast<long long>(nms_runs(bt.h)) * bt.bpr;
        rs += stack_floats(bt.h, bt.w, K);
    }
    __syncthreads();
    const bool valid = !bad_s && tot_pix <= max_pixels && tot_items * K < (1LL << 30) &&
                       tot_nms < (1LL << 30) && tot_mitems * K < (1LL << 30) &&
                       tot_nitems < (1LL << 30);
    if (threadIdx.x == 0) {
        ctr->items_per_scale = valid ? static_cast<int>(tot_items) : 0;
        ctr->nms_blocks = valid ? static_cast<int>(tot_nms) : 0;
        ctr->nms_items = valid ? static_cast<int>(tot_nitems) : 0;
        ctr->valid = valid ? 1 : 0;
        ctr->pool_used = 0;
        ctr->flags = 0;
        ctr->n_cand = 0;
        ctr->n_blobs = 0;
        ctr->work[0] = ctr->work[1] = ctr->work[2] = 0;
        ctr->mitems_per_scale = valid ? static_cast<int>(tot_mitems) : 0;
        for (int i = 0; i < MFMA_SHAPES; ++i) ctr->mwork[i] = 0;
    }
    if (!valid) {
        for (int t = t0; t < t1; ++t) {
            mhfd_result* r = in[t].result;
            if (r) {
                r->n_blobs = 0;
                r->n_candidates = 0;
                r->flags = MHFD_FLAG_INVALID_TILE;
                r->reserved = 0;
                r->density = 0.0;
            }
        }
    }
}

// Persistent maxima waves over every tile's (run of nms::ROWS rows, strip of
// 64 nms_cw columns) items, the per-wave body of the single-tile pass; the
// tile index rides in the upper bits of every record's k.
// Every index a wave derives its tile and cell from is wave-uniform
// (readfirstlane), so that bookkeeping stays in scalar registers: without it
// the kernel held 190 vector registers, with it 149 (three waves per SIMD);
// with the four-column path (K <= 10) it holds 229 (two waves per SIMD) and
// the 64-tile fp32 batch runs 3% faster.
template <int K, bool SPARSE>
__global__ __launch_bounds__(64 * NMS_WAVES) void nms_batch_kernel(
    const float* __restrict__ stack, const BatchTile* __restrict__ tiles, int n_tiles, float tau,
    int n_blk_bound, int32_t* __restrict__ blk_n, int32_t* __restrict__ blk_o,
    Cand* __restrict__ pool, int64_t cap, BatchCounters* __restrict__ ctr,
    const uint64_t* __restrict__ act) {
    const int total = ctr->nms_items;
    const int n_waves = gridDim.x * NMS_WAVES;

    // wave-uniform (readfirstlane), so the tile fields come in scalar
    // registers rather than in every lane's
    const int wave0 = __builtin_amdgcn_readfirstlane(blockIdx.x * NMS_WAVES + (threadIdx.x >> 6));
    // A wave's items increase, so its tile (the last t with nitem_base <=
    // item) only moves forward: one binary search, then a cursor.
    int lo = 0;
    {
        const int first = wave0;
        int hi = n_tiles;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tiles[mid].nitem_base <= first)
                lo = mid;
            else
                hi = mid;
        }
    }
    for (int item = wave0; item < total; item += n_waves) {
        while (lo + 1 < n_tiles && tiles[lo + 1].nitem_base <= item) ++lo;
        const BatchTile& T = tiles[lo];

        const int local = item - T.nitem_base;
        const int run = local / T.bpr, strip = local - run * T.bpr;
        nms::Sink out;
        out.blk_n = blk_n + T.nms_base;
        out.blk_o = blk_o + T.nms_base;
        out.slots = pool + static_cast<int64_t>(T.nms_base) * SLOT;
        out.over = pool + static_cast<int64_t>(n_blk_bound) * SLOT;
        out.cap = cap;
        out.pool_used = &ctr->pool_used;
        out.flags = &ctr->flags;
        out.k_tag = lo << TILE_SHIFT;
        const float* st = stack + T.stack_off;
        const nms::Active a{SPARSE ? act + T.act_off : nullptr, (T.w + 15) / 16, (T.h + 15) / 16};
        if constexpr (K <= 10) {
            if (T.nms_cw == 4) {
                nms::wave<K, 4, SLOT, SPARSE>(st, T.h, T.w, tau, T.bpr, strip, run, out, a);
                continue;
            }
        }
        if constexpr (2 * K <= 32) {
            if (T.nms_cw == 2) {
                nms::wave<K, 2, SLOT, SPARSE>(st, T.h, T.w, tau, T.bpr, strip, run, out, a);
                continue;
            }
        }
        nms::wave<K, 1, SLOT, SPARSE>(st, T.h, T.w, tau, T.bpr, strip, run, out, a);
    }
}

// Also sets every candidate's keep flag to 1 (the prune clears flags).
__global__ void order_batch_kernel(const int32_t* __restrict__ blk_off,
                                   const int32_t* __restrict__ blk_o, int n_blk_bound,
                                   const Cand* __restrict__ pool, Cand* __restrict__ cand,
                                   int32_t* __restrict__ keep, int64_t cap,
                                   BatchCounters* __restrict__ ctr) {
    const int n_blk = ctr->nms_blocks;
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    if (blockIdx.x == 0 && threadIdx.x == 0 && ctr->n_cand > cap)
        atomicOr(&ctr->flags, MHFD_FLAG_CAND_OVERFLOW);
    const Cand* over = pool + static_cast<int64_t>(n_blk_bound) * SLOT;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int lo = 0, hi = n_blk;
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

// Overlap prune over all tiles, one work item per (candidate, row offset)
// as in the single-tile path; rows are those of the candidate's own tile.
__global__ void prune_rows_batch_kernel(const Cand* __restrict__ cand,
                                        const int32_t* __restrict__ blk_off,
                                        const BatchTile* __restrict__ tiles, int K,
                                        const int32_t* __restrict__ d2max, int reach,
                                        int d2top, int32_t* __restrict__ keep, int64_t cap,
                                        const BatchCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    const long long dy = static_cast<long long>(blockIdx.y) - reach;
    const int xr = static_cast<int>(sqrt(static_cast<double>(d2top - dy * dy)));
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Cand b = cand[i];
        const int ti = b.k >> TILE_SHIFT, kb = b.k & ((1 << TILE_SHIFT) - 1);
        const BatchTile& T = tiles[ti];
        const long long yy = b.y + dy;
        if (yy < 0 || yy >= T.h || !keep[i]) continue;
        const int32_t* dcol = d2max + kb;
        int lo = blk_off[T.nms_base + yy * T.bpr];
        const int hi = min(static_cast<int64_t>(blk_off[T.nms_base + (yy + 1) * T.bpr]), n);
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
            const int ka = a.k & ((1 << TILE_SHIFT) - 1);
            const bool dom = ka > kb || (ka == kb && (a.y < b.y || (a.y == b.y && a.x < b.x)));
            const long long dx = a.x - b.x;
            if (dom && dy * dy + dx * dx <= dcol[ka * K]) {
                keep[i] = 0;
                break;
            }
        }
    }
}

__global__ void emit_batch_kernel(const Cand* __restrict__ cand, const int32_t* __restrict__ keep,
                                  const int32_t* __restrict__ keep_off,
                                  const int32_t* __restrict__ blk_off,
                                  const BatchTile* __restrict__ tiles,
                                  const float* __restrict__ sigmas, int64_t cap,
                                  const BatchCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (!keep[i]) continue;
        const Cand c = cand[i];
        const int ti = c.k >> TILE_SHIFT, k = c.k & ((1 << TILE_SHIFT) - 1);
        const BatchTile& T = tiles[ti];
        const int64_t first = blk_off[T.nms_base];  // first candidate of the tile
        const int pos = keep_off[i] - keep_off[first];
        if (pos < T.capacity) {
            mhfd_blob b;
            b.y = c.y;
            b.x = c.x;
            b.k = k;
            b.sigma = sigmas[k];
            b.response = c.r;
            T.blobs[pos] = b;
        }
    }
}

__global__ void results_batch_kernel(const int32_t* __restrict__ blk_off,
                                     const int32_t* __restrict__ keep_off,
                                     const BatchTile* __restrict__ tiles, int n_tiles, int64_t cap,
                                     const BatchCounters* __restrict__ ctr) {
    if (!ctr->valid) return;
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) {
        const BatchTile& T = tiles[t];
        const int64_t cb = blk_off[T.nms_base];
        const int64_t ce = blk_off[T.nms_base + T.h * T.bpr];
        const int64_t kb = keep_off[min(cb, n)], ke = keep_off[min(ce, n)];
        int32_t flags = ctr->flags & MHFD_FLAG_CAND_OVERFLOW;
        const int64_t nb = ke - kb;
        if (nb > T.capacity) flags |= MHFD_FLAG_BLOB_OVERFLOW;
        T.result->n_blobs = nb;
        T.result->n_candidates = ce - cb;
        T.result->flags = flags;
        T.result->reserved = 0;
        T.result->density = static_cast<double>(nb) * 1e6 / (static_cast<double>(T.h) * T.w);
    }
}

template <int K>
void launch_nms_batch_k(const BatchLaunchArgs& a, hipStream_t s) {
    if (a.act)
        nms_batch_kernel<K, true><<<a.nms_grid, 64 * NMS_WAVES, 0, s>>>(
            a.stack, a.tiles, a.n_tiles, a.tau, a.n_blk_bound, a.blk_n, a.blk_o, a.pool, a.cap,
            a.ctr, a.act);
    else
        nms_batch_kernel<K, false><<<a.nms_grid, 64 * NMS_WAVES, 0, s>>>(
            a.stack, a.tiles, a.n_tiles, a.tau, a.n_blk_bound, a.blk_n, a.blk_o, a.pool, a.cap,
            a.ctr, a.act);
}

template <int... Ks>
void launch_nms_batch(int K, const BatchLaunchArgs& a, hipStream_t s,
                      std::integer_sequence<int, Ks...>) {
    ((K == Ks + 1 ? launch_nms_batch_k<Ks + 1>(a, s) : void()), ...);
}

}  // namespace

hipError_t launch_batch_setup(const mhfd_tile* in, int n, long long max_pixels, int K, int max_h,
                              int max_w, int dtype, int mfma, BatchTile* tiles,
                              BatchCounters* ctr, hipStream_t s) {
    batch_setup_kernel<<<1, SETUP_T, 0, s>>>(in, n, max_pixels, K, max_h, max_w, dtype, mfma,
                                             tiles, ctr);
    return hipGetLastError();
}

hipError_t launch_batch_tail(const BatchLaunchArgs& a, hipStream_t s) {
    launch_nms_batch(a.K, a, s, std::make_integer_sequence<int, MHFD_MAX_SCALES>{});
    launch_batch_scan(a.blk_n, a.n_blk_bound, &a.ctr->nms_blocks, a.scan_sums, a.blk_off,
                      &a.ctr->n_cand, s);
    const int grid = 1024;
    order_batch_kernel<<<grid, 256, 0, s>>>(a.blk_off, a.blk_o, a.n_blk_bound, a.pool, a.cand,
                                            a.keep, a.cap, a.ctr);
    if (a.d2max) {
        const int span = 2 * a.reach + 1;
        prune_rows_batch_kernel<<<dim3(prune_grid_x(span), span), 256, 0, s>>>(
            a.cand, a.blk_off, a.tiles, a.K, a.d2max, a.reach, a.d2top, a.keep, a.cap, a.ctr);
    }
    launch_batch_scan(a.keep, static_cast<int>(a.cap), &a.ctr->n_cand, a.scan_sums, a.keep_off,
                      &a.ctr->n_blobs, s);
    emit_batch_kernel<<<grid, 256, 0, s>>>(a.cand, a.keep, a.keep_off, a.blk_off, a.tiles,
                                           a.sigmas, a.cap, a.ctr);
    results_batch_kernel<<<(a.n_tiles + 255) / 256, 256, 0, s>>>(a.blk_off, a.keep_off, a.tiles,
                                                                 a.n_tiles, a.cap, a.ctr);
    return hipGetLastError();
}

}  // namespace mhfd
