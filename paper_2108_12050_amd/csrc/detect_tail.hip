// Detection after the LoG stack: 3x3x3 maxima, threshold, compaction into
// canonical (y, x, k) order, one-shot overlap pruning, blob list.
//
//   nms        one workgroup per (row, 256-column chunk).  A thread owns one
//              pixel and walks the scales keeping the 3x3 spatial maxima of
//              planes k-1, k, k+1; vertical maxima are shared through LDS.
//              A voxel is a candidate when it equals the maximum of its
//              3x3x3 window (the maxpool-equality test of section 3, taken
//              local in scale too) and is above the threshold.  Counts per
//              thread become in-wave offsets with ballot + mbcnt over the
//              bits of the count; each workgroup reserves one run in an
//              unordered pool with a single atomic.
//   scan       exclusive scan of the per-workgroup counts in workgroup order,
//              i.e. in (y, x) order: the canonical position of every run.
//   order      copies each run from the pool to its canonical place.
//   prune      one thread per candidate scans the candidates of the rows
//              that can reach it (row ranges come from the scan) and applies
//              the dominance rule with FP64 lens geometry.
//   emit       scan of the keep flags, then the blob records.
// No step depends on the order in which workgroups run, so the output is
// deterministic.
#include <float.h>
#include <math.h>

#include <utility>

#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int NMS_T = 256;
constexpr int SLOT = 16;  // pool records each NMS workgroup owns
constexpr int SCAN_T = 1024;

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

__global__ void init_counters_kernel(DetectCounters* ctr) {
    if (threadIdx.x == 0) {
        ctr->pool_used = 0;
        ctr->flags = 0;
        ctr->n_cand = 0;
        ctr->n_blobs = 0;
    }
}

// One workgroup per (row, 256-column chunk).  Every thread first issues the
// loads of its column's three rows for all K planes: indices are clamped so
// that every load is in bounds and unconditional (no branch, so all 3K loads
// are in flight together), and values from outside the image are replaced by
// -inf afterwards.  Vertical 3-maxima go through LDS once, then each thread
// tests its K voxels.
template <int K>
__global__ __launch_bounds__(NMS_T) void nms_kernel(const float* __restrict__ st, int H, int W,
                                                    float tau, int bpr,
                                                    int32_t* __restrict__ blk_n,
                                                    int32_t* __restrict__ blk_o,
                                                    Cand* __restrict__ pool, int64_t cap,
                                                    DetectCounters* __restrict__ ctr) {
    __shared__ float vm[K][NMS_T + 2];
    __shared__ int wave_tot[NMS_T / 64];
    __shared__ int run_base;

    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int y = blk / bpr;
    const int x0 = (blk - y * bpr) * NMS_T;
    const int x = x0 + tid;
    const bool valid = x < W;
    const size_t plane = static_cast<size_t>(H) * W;
    const int yu = y > 0 ? y - 1 : 0;
    const int yd = y + 1 < H ? y + 1 : H - 1;
    const int xc = valid ? x : W - 1;

    float cv[K], vmx[K];
    {
        const float* pc = st + static_cast<size_t>(y) * W + xc;
        const float* pu = st + static_cast<size_t>(yu) * W + xc;
        const float* pd = st + static_cast<size_t>(yd) * W + xc;
        float u[K], d[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            cv[k] = pc[k * plane];
            u[k] = pu[k * plane];
            d[k] = pd[k * plane];
        }
        // rows clamped onto the centre row contribute nothing new to the max
#pragma unroll
        for (int k = 0; k < K; ++k) vmx[k] = valid ? fmax3(u[k], cv[k], d[k]) : -INFINITY;
    }
    // halo columns x0 - 1 and x0 + 256 (clamped, then masked)
    if (tid == 0 || tid == NMS_T - 1) {
        const int xh = tid == 0 ? x0 - 1 : x0 + NMS_T;
        const bool ok = xh >= 0 && xh < W;
        const int xs = ok ? xh : 0;
        const int slot = tid == 0 ? 0 : NMS_T + 1;
        const float* pc = st + static_cast<size_t>(y) * W + xs;
        const float* pu = st + static_cast<size_t>(yu) * W + xs;
        const float* pd = st + static_cast<size_t>(yd) * W + xs;
        float hv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) hv[k] = fmax3(pu[k * plane], pc[k * plane], pd[k * plane]);
#pragma unroll
        for (int k = 0; k < K; ++k) vm[k][slot] = ok ? hv[k] : -INFINITY;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) vm[k][tid + 1] = vmx[k];
    __syncthreads();

    unsigned mask = 0u;
    {
        float m_prev = -INFINITY;
        float m_cur = fmax3(vm[0][tid], vm[0][tid + 1], vm[0][tid + 2]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float m_next =
                k + 1 < K ? fmax3(vm[k + 1][tid], vm[k + 1][tid + 1], vm[k + 1][tid + 2]) : -INFINITY;
            const float v = cv[k];
            if (v > tau && v >= fmax3(m_prev, m_cur, m_next)) mask |= 1u << k;
            m_prev = m_cur;
            m_cur = m_next;
        }
        if (!valid) mask = 0u;
    }

    const int c = __popc(mask);
    int wtot;
    const int pre = wave_exclusive_prefix<6>(c, &wtot);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) wave_tot[wv] = wtot;
    __syncthreads();
    int woff = 0, n = 0;
#pragma unroll
    for (int i = 0; i < NMS_T / 64; ++i) {
        woff += i < wv ? wave_tot[i] : 0;
        n += wave_tot[i];
    }
    // The first SLOT records of a workgroup go to its own pool slot; a
    // workgroup with more reserves room for the rest in the shared overflow
    // region (one atomic, only for such workgroups).
    if (tid == 0) {
        int o = 0;
        if (n > SLOT) {
            o = atomicAdd(&ctr->pool_used, n - SLOT);
            if (static_cast<int64_t>(o) + (n - SLOT) > cap)
                atomicOr(&ctr->flags, MHFD_FLAG_CAND_OVERFLOW);
        }
        run_base = o;
        blk_n[blk] = n;
        blk_o[blk] = o;
    }
    __syncthreads();
    if (c > 0) {
        int j = woff + pre;  // rank of this thread's first record in the workgroup
        Cand* own = pool + static_cast<int64_t>(blk) * SLOT;
        Cand* over = pool + static_cast<int64_t>(gridDim.x) * SLOT + run_base - SLOT;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (mask & (1u << k)) {
                Cand r;
                r.y = y;
                r.x = x;
                r.k = k;
                r.r = cv[k];
                if (j < SLOT)
                    own[j] = r;
                else if (run_base + (j - SLOT) < cap)
                    over[j] = r;
                ++j;
            }
        }
    }
}

template <int K>
void launch_nms_k(const DetectWorkspace& ws, int h, int w, float tau, hipStream_t s) {
    nms_kernel<K><<<ws.n_blk, NMS_T, 0, s>>>(ws.stack, h, w, tau, ws.blk_per_row, ws.blk_n,
                                             ws.blk_o, ws.pool, ws.cap, ws.ctr);
}

template <int... Ks>
void launch_nms(int K, const DetectWorkspace& ws, int h, int w, float tau, hipStream_t s,
                std::integer_sequence<int, Ks...>) {
    ((K == Ks + 1 ? launch_nms_k<Ks + 1>(ws, h, w, tau, s) : void()), ...);
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

void launch_scan(const int32_t* in, int n_host, const int32_t* n_dev, int32_t* sums,
                 int32_t* out, int32_t* total_out, hipStream_t s) {
    const int nb = (n_host + SCAN_SPAN - 1) / SCAN_SPAN;
    const int grid = nb > 0 ? nb : 1;
    scan_sums_kernel<<<grid, SCAN_BT, 0, s>>>(in, n_host, n_dev, sums);
    scan_top_kernel<<<1, 1024, 0, s>>>(sums, grid, n_host, n_dev, out, total_out);
    scan_apply_kernel<<<grid, SCAN_BT, 0, s>>>(in, n_host, n_dev, sums, out);
}

__global__ void order_kernel(const int32_t* __restrict__ blk_off, const int32_t* __restrict__ blk_o,
                             int n_blk, const Cand* __restrict__ pool, Cand* __restrict__ cand,
                             int64_t cap, const DetectCounters* __restrict__ ctr) {
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
    }
}

// One thread per candidate b.  Candidates a that can remove b lie within
// `reach` rows and, in row y_b + dy, within |dx| <= sqrt(reach^2 - dy^2);
// rows come from the per-row offsets of the canonical list and the column
// range from a binary search in the row (sorted by x).  The overlap test is
// the plan's exact integer form: overlap(a, b) > theta iff
// dy^2 + dx^2 <= d2max[k_a][k_b] (the lens fraction falls monotonically with
// distance; the table is evaluated in double on the host).
__global__ void prune_kernel(const Cand* __restrict__ cand, const int32_t* __restrict__ blk_off,
                             int bpr, int H, int K, const int32_t* __restrict__ d2max, int reach,
                             int32_t* __restrict__ keep, int64_t cap,
                             const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    const long long r2 = static_cast<long long>(reach) * reach;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Cand b = cand[i];
        const int32_t* dcol = d2max + b.k;  // d2max[ka * K + kb]
        int kp = 1;
        const int ylo = max(0, b.y - reach), yhi = min(H - 1, b.y + reach);
        for (int yy = ylo; yy <= yhi && kp; ++yy) {
            const long long dy = yy - b.y;
            const int xr = static_cast<int>(sqrt(static_cast<double>(r2 - dy * dy)));
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
                const bool dom =
                    a.k > b.k || (a.k == b.k && (a.y < b.y || (a.y == b.y && a.x < b.x)));
                const long long dx = a.x - b.x;
                if (dom && dy * dy + dx * dx <= dcol[a.k * K]) {
                    kp = 0;
                    break;
                }
            }
        }
        keep[i] = kp;
    }
}

__global__ void keep_all_kernel(int32_t* __restrict__ keep, int64_t cap,
                                const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        keep[i] = 1;
}

__global__ void emit_kernel(const Cand* __restrict__ cand, const int32_t* __restrict__ keep,
                            const int32_t* __restrict__ keep_off, const float* __restrict__ sigmas,
                            mhfd_blob* __restrict__ blobs, int capacity, int64_t cap,
                            DetectCounters* __restrict__ ctr, mhfd_result* __restrict__ result) {
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
    }
}

}  // namespace

int nms_blocks_per_row(int w) { return (w + NMS_T - 1) / NMS_T; }

void launch_batch_scan(const int32_t* in, int n_host, const int32_t* n_dev, int32_t* sums,
                       int32_t* out, int32_t* total_out, hipStream_t s) {
    launch_scan(in, n_host, n_dev, sums, out, total_out, s);
}

size_t nms_pool_records(int n_blk, int64_t cap) { return static_cast<size_t>(n_blk) * SLOT + cap; }

size_t scan_sums_ints(int64_t n) { return static_cast<size_t>((n + SCAN_SPAN - 1) / SCAN_SPAN + 1); }

hipError_t launch_detect_tail(const DetectWorkspace& ws, int K, int h, int w, float tau,
                              const int32_t* d2max, int reach, const float* sigmas_dev,
                              mhfd_blob* blobs, int capacity, mhfd_result* result, hipStream_t s) {
    init_counters_kernel<<<1, 64, 0, s>>>(ws.ctr);
    launch_nms(K, ws, h, w, tau, s, std::make_integer_sequence<int, MHFD_MAX_SCALES>{});
    launch_scan(ws.blk_n, ws.n_blk, nullptr, ws.scan_sums, ws.blk_off, &ws.ctr->n_cand, s);
    const int grid = 1024;
    order_kernel<<<grid, 256, 0, s>>>(ws.blk_off, ws.blk_o, ws.n_blk, ws.pool, ws.cand, ws.cap,
                                      ws.ctr);
    if (d2max)
        prune_kernel<<<grid, 256, 0, s>>>(ws.cand, ws.blk_off, ws.blk_per_row, h, K, d2max, reach,
                                          ws.keep, ws.cap, ws.ctr);
    else
        keep_all_kernel<<<grid, 256, 0, s>>>(ws.keep, ws.cap, ws.ctr);
    launch_scan(ws.keep, static_cast<int>(ws.cap), &ws.ctr->n_cand, ws.scan_sums, ws.keep_off,
                &ws.ctr->n_blobs, s);
    emit_kernel<<<grid, 256, 0, s>>>(ws.cand, ws.keep, ws.keep_off, sigmas_dev, blobs, capacity,
                                     ws.cap, ws.ctr, result);
    return hipGetLastError();
}

}  // namespace mhfd
