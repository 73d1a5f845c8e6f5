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

#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int NMS_T = 256;
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

__global__ __launch_bounds__(NMS_T) void nms_kernel(const float* __restrict__ st, int K, int H,
                                                    int W, float tau, int bpr,
                                                    int32_t* __restrict__ blk_n,
                                                    int32_t* __restrict__ blk_o,
                                                    Cand* __restrict__ pool, int64_t cap,
                                                    DetectCounters* __restrict__ ctr) {
    __shared__ float vm[2][NMS_T + 2];
    __shared__ int wave_tot[NMS_T / 64];
    __shared__ int run_base;

    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int y = blk / bpr;
    const int x0 = (blk - y * bpr) * NMS_T;
    const int x = x0 + tid;
    const bool valid = x < W;
    const size_t plane = static_cast<size_t>(H) * W;

    // Largest of rows y-1..y+1 of plane k at column xc, -inf outside.
    auto vmax = [&](int k, int xc) -> float {
        if (xc < 0 || xc >= W) return -INFINITY;
        const float* p = st + k * plane + static_cast<size_t>(y) * W + xc;
        float m = p[0];
        if (y > 0) m = fmaxf(m, p[-W]);
        if (y + 1 < H) m = fmaxf(m, p[W]);
        return m;
    };

    float m_prev2 = -INFINITY, m_prev = -INFINITY, v_prev = -INFINITY;
    unsigned long long mask = 0ull;
    for (int k = 0; k <= K; ++k) {
        const int buf = k & 1;
        if (k < K) {
            vm[buf][tid + 1] = vmax(k, x);
            if (tid == 0) vm[buf][0] = vmax(k, x0 - 1);
            if (tid == NMS_T - 1) vm[buf][NMS_T + 1] = vmax(k, x0 + NMS_T);
        }
        __syncthreads();
        float m_cur = -INFINITY, v_cur = -INFINITY;
        if (k < K && valid) {
            m_cur = fmax3(vm[buf][tid], vm[buf][tid + 1], vm[buf][tid + 2]);
            v_cur = st[k * plane + static_cast<size_t>(y) * W + x];
        }
        if (k >= 1 && valid) {
            const float mm = fmax3(m_prev2, m_prev, m_cur);
            if (v_prev > tau && v_prev >= mm) mask |= 1ull << (k - 1);
        }
        m_prev2 = m_prev;
        m_prev = m_cur;
        v_prev = v_cur;
    }

    const int c = __popcll(mask);
    int wtot;
    const int pre = wave_exclusive_prefix<7>(c, &wtot);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) wave_tot[wv] = wtot;
    __syncthreads();
    int woff = 0, n = 0;
#pragma unroll
    for (int i = 0; i < NMS_T / 64; ++i) {
        woff += i < wv ? wave_tot[i] : 0;
        n += wave_tot[i];
    }
    if (tid == 0) {
        int o = 0;
        if (n > 0) {
            o = atomicAdd(&ctr->pool_used, n);
            if (static_cast<int64_t>(o) + n > cap) atomicOr(&ctr->flags, MHFD_FLAG_CAND_OVERFLOW);
        }
        run_base = o;
        blk_n[blk] = n;
        blk_o[blk] = o;
    }
    __syncthreads();
    if (c > 0) {
        int64_t pos = static_cast<int64_t>(run_base) + woff + pre;
        unsigned long long m = mask;
        while (m) {
            const int k = __ffsll(m) - 1;
            m &= m - 1;
            if (pos < cap) {
                Cand r;
                r.y = y;
                r.x = x;
                r.k = k;
                r.r = st[k * plane + static_cast<size_t>(y) * W + x];
                pool[pos] = r;
            }
            ++pos;
        }
    }
}

// Exclusive scan of in[0, n) into out[0, n], out[n] = total, by one
// workgroup.  n is min(n_host, *n_dev) when n_dev is given.  If total_out is
// given it receives the total as well.
__global__ __launch_bounds__(SCAN_T) void scan_kernel(const int32_t* __restrict__ in, int n_host,
                                                      const int32_t* __restrict__ n_dev,
                                                      int32_t* __restrict__ out,
                                                      int32_t* __restrict__ total_out) {
    __shared__ int part[SCAN_T];
    int n = n_host;
    if (n_dev) n = min(n, *n_dev);
    const int tid = threadIdx.x;
    const int per = (n + SCAN_T - 1) / SCAN_T;
    const int lo = min(n, tid * per), hi = min(n, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the partial sums
    for (int d = 1; d < SCAN_T; d <<= 1) {
        const int v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        out[i] = run;
        run += in[i];
    }
    if (tid == SCAN_T - 1) {
        out[n] = part[SCAN_T - 1];
        if (total_out) *total_out = part[SCAN_T - 1];
    }
}

__global__ void order_kernel(const int32_t* __restrict__ blk_off, const int32_t* __restrict__ blk_o,
                             int n_blk, const Cand* __restrict__ pool, Cand* __restrict__ cand,
                             int64_t cap, const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        // last block b with blk_off[b] <= i
        int lo = 0, hi = n_blk;  // invariant: blk_off[lo] <= i < blk_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (blk_off[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t src = static_cast<int64_t>(blk_o[lo]) + (i - blk_off[lo]);
        if (src < cap) cand[i] = pool[src];
    }
}

// Fraction of the smaller disc covered by the intersection of two discs.
__device__ double disc_overlap(double dy, double dx, double ra, double rb) {
    const double d = sqrt(dy * dy + dx * dx);
    if (d >= ra + rb) return 0.0;
    if (d <= fabs(ra - rb)) return 1.0;
    const double rs = fmin(ra, rb);
    const double ca = (d * d + ra * ra - rb * rb) / (2.0 * d * ra);
    const double cb = (d * d + rb * rb - ra * ra) / (2.0 * d * rb);
    const double lens = ra * ra * acos(ca) + rb * rb * acos(cb) -
                        0.5 * sqrt((-d + ra + rb) * (d + ra - rb) * (d - ra + rb) * (d + ra + rb));
    return lens / (M_PI * rs * rs);
}

__global__ void prune_kernel(const Cand* __restrict__ cand, const int32_t* __restrict__ blk_off,
                             int bpr, int H, const float* __restrict__ sigmas, int reach,
                             double theta, int32_t* __restrict__ keep, int64_t cap,
                             const DetectCounters* __restrict__ ctr) {
    const int64_t n = min(static_cast<int64_t>(ctr->n_cand), cap);
    const double kSqrt2 = 1.4142135623730951;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Cand b = cand[i];
        const double rb = kSqrt2 * static_cast<double>(sigmas[b.k]);
        const int ylo = max(0, b.y - reach), yhi = min(H - 1, b.y + reach);
        const int64_t j0 = blk_off[ylo * bpr];
        const int64_t j1 = min(static_cast<int64_t>(blk_off[(yhi + 1) * bpr]), n);
        int kp = 1;
        for (int64_t j = j0; j < j1 && kp; ++j) {
            if (j == i) continue;
            const Cand a = cand[j];
            const bool dom = a.k > b.k || (a.k == b.k && (a.y < b.y || (a.y == b.y && a.x < b.x)));
            if (!dom) continue;
            const double ra = kSqrt2 * static_cast<double>(sigmas[a.k]);
            const double dy = static_cast<double>(a.y - b.y), dx = static_cast<double>(a.x - b.x);
            if (fabs(dx) >= ra + rb) continue;  // disjoint discs (overlap 0)
            if (disc_overlap(dy, dx, ra, rb) > theta) kp = 0;
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

hipError_t launch_detect_tail(const DetectWorkspace& ws, int K, int h, int w, float tau,
                              float overlap, int reach, const float* sigmas_dev, mhfd_blob* blobs,
                              int capacity, mhfd_result* result, hipStream_t s) {
    init_counters_kernel<<<1, 64, 0, s>>>(ws.ctr);
    nms_kernel<<<ws.n_blk, NMS_T, 0, s>>>(ws.stack, K, h, w, tau, ws.blk_per_row, ws.blk_n,
                                          ws.blk_o, ws.pool, ws.cap, ws.ctr);
    scan_kernel<<<1, SCAN_T, 0, s>>>(ws.blk_n, ws.n_blk, nullptr, ws.blk_off, &ws.ctr->n_cand);
    const int grid = 1024;
    order_kernel<<<grid, 256, 0, s>>>(ws.blk_off, ws.blk_o, ws.n_blk, ws.pool, ws.cand, ws.cap,
                                      ws.ctr);
    if (overlap < 1.0f) {
        prune_kernel<<<grid, 256, 0, s>>>(ws.cand, ws.blk_off, ws.blk_per_row, h, sigmas_dev,
                                          reach, static_cast<double>(overlap), ws.keep, ws.cap,
                                          ws.ctr);
    } else {
        keep_all_kernel<<<grid, 256, 0, s>>>(ws.keep, ws.cap, ws.ctr);
    }
    scan_kernel<<<1, SCAN_T, 0, s>>>(ws.keep, static_cast<int>(ws.cap), &ws.ctr->n_cand,
                                     ws.keep_off, &ws.ctr->n_blobs);
    emit_kernel<<<grid, 256, 0, s>>>(ws.cand, ws.keep, ws.keep_off, sigmas_dev, blobs, capacity,
                                     ws.cap, ws.ctr, result);
    return hipGetLastError();
}

}  // namespace mhfd
