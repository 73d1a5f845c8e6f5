// Scale-normalised LoG stack, streamed down vertical strips.
//
// R_k = s sigma_k^2 (h (*)_y A + g (*)_y B),  A = g (*)_x I,  B = h (*)_x I
// (the 2-D Gaussian of section 2.2 factorises as g(x) g(y), so its Laplacian
// is h(x) g(y) + g(x) h(y)).  Every scale is independent of the others
// (section 3 makes the same observation for the per-scale filtering): one
// launch covers every scale of a radius class, each workgroup owning one
// (scale, strip, segment); scales run largest radius first so the longest
// workgroups start first.
//
// A workgroup owns a strip of TW output columns and a segment of rows of one
// scale.  It walks down the segment in chunks of CH rows:
//   stage   CH input rows, columns [x0 - R, x0 + TW + R), into LDS, with the
//           half-sample reflection at the image borders.  The global loads
//           of chunk m+1 are issued into registers before the passes of
//           chunk m, so their latency hides behind arithmetic;
//   row     pass: A and B of those rows (TW columns) into an LDS ring that
//           holds the last CH + 2R rows, so every row pass is done once per
//           segment and not once per output tile;
//   column  pass: CH output rows from the ring, with the Laplacian sum and the
//           s sigma^2 factor folded into the column taps; written to HBM.
// The row pass keeps 8 + 2R input values of one row in registers and forms
// 8 outputs from symmetric pair sums (one add feeds both the g and the h
// product).  The column pass keeps 8 + 2R ring values of one column in
// registers and forms 8 output rows, first from the A ring, then from the B
// ring.  Both loop over taps outermost, so the wave-uniform taps stream
// through scalar registers.
#include "mhfd_internal.h"

namespace mhfd {

namespace {

constexpr int TW = 64;   // output columns per strip (one per lane in the column pass)
constexpr int CH = 32;   // rows per chunk
constexpr int NT = 256;  // threads per workgroup (4 waves)
constexpr int PX = 8;    // row-pass outputs per thread
constexpr int QY = 8;    // column-pass outputs per thread
constexpr int TAP_BATCH = 16;  // taps whose loads may be in flight together

static_assert(NT / 8 == CH, "row pass: 8 threads per row, one row per thread group");
static_assert(TW == 8 * PX, "row pass: 8 threads cover the strip");
static_assert((NT / 64) * QY == CH, "column pass: one wave per 8 rows");

__host__ __device__ constexpr int lds_floats(int R) {
    return CH * (TW + 2 * R) + 2 * (CH + 2 * R) * TW;  // input chunk, A ring, B ring
}

// taps + j0 through an offset the compiler cannot see through.  Without it
// the compiler hoists every tap load of the kernel out of the chunk loop
// and keeps 4(R + 1) taps in scalar registers, more than the scalar file
// holds; the excess is spilled to vector lanes and read back with one extra
// vector instruction per use.  With it, one batch of taps is live at a time,
// fetched by wide scalar loads that hit the scalar cache.
__device__ __forceinline__ const float* tap_block(const float* __restrict__ taps, int j0) {
    int o = j0;
    asm volatile("" : "+s"(o));
    return taps + o;
}

__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(uint8_t v) { return static_cast<float>(v) / 255.0f; }

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

// Block sum of one double per thread (fixed tree order); smem must hold NT doubles.
__device__ __forceinline__ double block_sum(double v, double* smem) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
    if ((threadIdx.x & 63) == 0) smem[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t += smem[i];
    return t;  // valid in thread 0
}

template <int R, int EPI, typename T>
__device__ __forceinline__ void log_strip_body(float* __restrict__ smem, const T* __restrict__ img,
                                               int H, int W, long long pitch,
                                               const float* __restrict__ taps,
                                               float* __restrict__ out, long long out_pitch,
                                               int x0, int ys, int ye, float beta, float tau,
                                               double* __restrict__ partial) {
    constexpr int NB = TW + 2 * R;            // staged input columns
    constexpr int S = CH + 2 * R;             // ring rows
    constexpr int P = (2 * R + CH - 1) / CH;  // prologue chunks (rows ys - R .. ys + R)
    static_assert(R % 4 == 0, "padded radius");
    float* in_s = smem;
    float* a_s = smem + CH * NB;   // ring of A rows, S x TW
    float* b_s = a_s + S * TW;     // ring of B rows, S x TW

    const int tid = threadIdx.x;
    const bool interior_x = (x0 - R >= 0) && (x0 + TW + R <= W);

    // Staging: wave w loads rows 8w .. 8w + 7 of a chunk; lane l loads columns
    // l, l + 64, ... of each row (coalesced), i.e. NG column groups whose image
    // columns (reflected at the borders) are fixed for the whole segment.
    constexpr int NG = (NB + 63) / 64;
    const int lane = tid & 63;
    const int wrow = __builtin_amdgcn_readfirstlane(tid >> 6) * (CH / 4);
    int gx[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int c = min(g * 64 + lane, NB - 1);
        gx[g] = interior_x ? x0 - R + c : reflect_index(x0 - R + c, W);
    }
    // First image row of staged chunk m, and its number of useful rows.
    auto chunk_r0 = [&](int m) { return m < P ? ys - R + m * CH : ys + R + (m - P) * CH; };
    auto chunk_n = [&](int m) { return m < P ? min(CH, 2 * R - m * CH) : CH; };

    T pf[CH / 4][NG];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int i = 0; i < CH / 4; ++i) {
            const long long rowoff = static_cast<long long>(reflect_index(r0 + wrow + i, H)) * pitch;
#pragma unroll
            for (int g = 0; g < NG; ++g) pf[i][g] = img[rowoff + gx[g]];
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int i = 0; i < CH / 4; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g)
                if (g * 64 + lane < NB) in_s[(wrow + i) * NB + g * 64 + lane] = to_float(pf[i][g]);
    };

    // A, B of rows [r0, r0 + n) into the ring; ring slot of row r: (r - ys + R) mod S.
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
            {
                const float* tp = tap_block(taps, 0);
                const float g0 = tp[0], h0 = tp[R + 1];
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    a[p] = g0 * v[p + R];
                    b[p] = h0 * v[p + R];
                }
            }
#pragma unroll
            for (int j0 = 1; j0 <= R; j0 += TAP_BATCH) {
                const float* tp = tap_block(taps, j0);  // g_row[j0] at tp[0], h_row[j0] at tp[R+1]
#pragma unroll
                for (int j = j0; j < j0 + TAP_BATCH && j <= R; ++j) {
                    const float gj = tp[j - j0];
                    const float hj = tp[(R + 1) + j - j0];
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        const float sum = v[p + R - j] + v[p + R + j];
                        a[p] = fmaf(gj, sum, a[p]);
                        b[p] = fmaf(hj, sum, b[p]);
                    }
                }
            }
            const int slot = (r0 + row - ys + R) % S;
            float4* da = reinterpret_cast<float4*>(a_s + slot * TW + cg * PX);
            float4* db = reinterpret_cast<float4*>(b_s + slot * TW + cg * PX);
            da[0] = make_float4(a[0], a[1], a[2], a[3]);
            da[1] = make_float4(a[4], a[5], a[6], a[7]);
            db[0] = make_float4(b[0], b[1], b[2], b[3]);
            db[1] = make_float4(b[4], b[5], b[6], b[7]);
        }
    };

    float tsum = 0.0f;  // softplus sum of this thread's outputs (EPI_SOFTSUM)

    // Output rows [yc, yc + CH): wave w owns rows yc + 8w .. yc + 8w + 7, lane = column.
    // Two half passes, h (*)_y A then g (*)_y B, so only one 8 + 2R window of
    // ring values is live in registers at a time.
    auto colpass = [&](int yc) {
        const int q0 = __builtin_amdgcn_readfirstlane(tid >> 6) * QY;
        const int base = (yc + q0 - ys) % S;  // ring slot of image row yc + q0 - R
        float acc[QY];
#pragma unroll
        for (int q = 0; q < QY; ++q) acc[q] = 0.0f;
        auto half = [&](const float* ring, int tap0) {
            float win[QY + 2 * R];
#pragma unroll
            for (int t = 0; t < QY + 2 * R; ++t) {
                int slot = base + t;
                slot = slot >= S ? slot - S : slot;
                win[t] = ring[slot * TW + lane];
            }
            {
                const float c0 = tap_block(taps, tap0)[0];
#pragma unroll
                for (int q = 0; q < QY; ++q) acc[q] = fmaf(c0, win[q + R], acc[q]);
            }
#pragma unroll
            for (int a0 = 1; a0 <= R; a0 += TAP_BATCH) {
                const float* tp = tap_block(taps, tap0 + a0);
#pragma unroll
                for (int a = a0; a < a0 + TAP_BATCH && a <= R; ++a) {
                    const float c = tp[a - a0];
#pragma unroll
                    for (int q = 0; q < QY; ++q)
                        acc[q] = fmaf(c, win[q + R - a] + win[q + R + a], acc[q]);
                }
            }
        };
        half(a_s, 3 * (R + 1));  // h_col with A
        // keep the B window's loads behind the A half: overlapping the two
        // windows would double the live registers and halve occupancy
        __builtin_amdgcn_sched_barrier(0);
        half(b_s, 2 * (R + 1));  // g_col with B
        const int x = x0 + lane;
        if (x < W) {
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int y = yc + q0 + q;
                if (y < ye) {
                    float* o = out + static_cast<long long>(y) * out_pitch + x;
                    if constexpr (EPI == EPI_STORE) *o = acc[q];
                    if constexpr (EPI == EPI_ACCUM) *o += acc[q];
                    if constexpr (EPI == EPI_SOFTSUM) tsum += softplusf(beta * (fabsf(acc[q]) - tau));
                }
            }
        }
    };

    const int n_chunks = P + (ye - ys + CH - 1) / CH;
    fetch(chunk_r0(0));
    for (int m = 0; m < n_chunks; ++m) {
        commit();
        __syncthreads();  // in_s holds chunk m; every wave is past the last column pass
        if (m + 1 < n_chunks) fetch(chunk_r0(m + 1));
        rowpass(chunk_r0(m), chunk_n(m));
        __syncthreads();
        if (m >= P) colpass(ys + (m - P) * CH);
    }
    if constexpr (EPI == EPI_SOFTSUM) {
        __syncthreads();  // smem is reused for the reduction
        const double t = block_sum(static_cast<double>(tsum), reinterpret_cast<double*>(smem));
        if (threadIdx.x == 0) *partial = t;
    }
}

// Radius classes share a kernel: registers are allocated for the largest
// radius of the class, so small radii do not pay for large ones.  blockIdx.y
// is the image of a batch.
template <int RLO, int RHI, int EPI, typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void log_stack_kernel(const T* __restrict__ img, int H, int W, long long pitch,
                      const float* __restrict__ taps, StackLaunch L, StackIO io) {
    extern __shared__ __attribute__((aligned(16))) float smem[];
    const int b = blockIdx.x;
    int i = 0;
    while (i + 1 < L.n && b >= L.sc[i + 1].block_begin) ++i;
    const StackScale sc = L.sc[i];
    const int local = b - sc.block_begin;
    const int strip = local % L.strips;
    const int seg = local / L.strips;
    const int x0 = strip * TW;
    const int ys = seg * sc.seg_rows;
    const int ye = min(ys + sc.seg_rows, H);
    const int bi = blockIdx.y;
    const T* im = img + static_cast<long long>(bi) * io.img_batch;
    float* out = io.out ? io.out + static_cast<long long>(bi) * io.out_batch +
                              static_cast<long long>(sc.plane) * io.plane_stride
                        : nullptr;
    double* part = io.partial ? io.partial + static_cast<long long>(bi) * io.total_blocks + b
                              : nullptr;
    const float* tp = taps + sc.tap_off;
    switch (sc.radius) {
#define MHFD_BODY(R)                                                                       \
    case R:                                                                                \
        if constexpr (R >= RLO && R <= RHI)                                                \
            log_strip_body<R, EPI, T>(smem, im, H, W, pitch, tp, out, W, x0, ys, ye,      \
                                      io.beta, io.tau, part);                              \
        break;
        MHFD_BODY(4)
        MHFD_BODY(8)
        MHFD_BODY(12)
        MHFD_BODY(16)
        MHFD_BODY(20)
        MHFD_BODY(24)
        MHFD_BODY(28)
        MHFD_BODY(32)
        MHFD_BODY(36)
        MHFD_BODY(40)
        MHFD_BODY(44)
        MHFD_BODY(48)
        MHFD_BODY(52)
        MHFD_BODY(56)
        MHFD_BODY(60)
        MHFD_BODY(64)
#undef MHFD_BODY
        default:
            break;
    }
}

template <int RLO, int RHI, int EPI, typename T>
hipError_t launch_typed(const T* img, int h, int w, int64_t pitch, int batch, const float* taps,
                        const StackLaunch& L, const StackIO& io, int blocks, size_t lds,
                        hipStream_t s) {
    auto k = log_stack_kernel<RLO, RHI, EPI, T>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    k<<<dim3(blocks, batch), NT, lds, s>>>(img, h, w, pitch, taps, L, io);
    return hipGetLastError();
}

template <int RLO, int RHI>
hipError_t launch_range(int in_dtype, int epi, const void* img, int h, int w, int64_t pitch,
                        int batch, const float* taps, const StackLaunch& L, const StackIO& io,
                        int blocks, size_t lds, hipStream_t s) {
    if (in_dtype == MHFD_U8) {
        if (epi != EPI_STORE) return hipErrorInvalidValue;
        return launch_typed<RLO, RHI, EPI_STORE, uint8_t>(static_cast<const uint8_t*>(img), h, w,
                                                          pitch, batch, taps, L, io, blocks, lds, s);
    }
    const float* f = static_cast<const float*>(img);
    if (epi == EPI_STORE)
        return launch_typed<RLO, RHI, EPI_STORE, float>(f, h, w, pitch, batch, taps, L, io, blocks,
                                                        lds, s);
    if (epi == EPI_ACCUM)
        return launch_typed<RLO, RHI, EPI_ACCUM, float>(f, h, w, pitch, batch, taps, L, io, blocks,
                                                        lds, s);
    return launch_typed<RLO, RHI, EPI_SOFTSUM, float>(f, h, w, pitch, batch, taps, L, io, blocks,
                                                      lds, s);
}

}  // namespace

int log_radius_class(int padded) { return padded <= 16 ? 0 : (padded <= 40 ? 1 : 2); }

int log_strip_width() { return TW; }

int log_chunk_rows() { return CH; }

hipError_t launch_log_class(int cls, int in_dtype, int epi, const void* img, int h, int w,
                            int64_t pitch, int batch, const float* taps, const StackLaunch& L,
                            const StackIO& io, hipStream_t s) {
    int blocks = 0, rmax = 0;
    for (int i = 0; i < L.n; ++i) {
        blocks += L.sc[i].n_blocks;
        rmax = L.sc[i].radius > rmax ? L.sc[i].radius : rmax;
    }
    if (blocks == 0 || batch == 0) return hipSuccess;
    size_t lds = sizeof(float) * static_cast<size_t>(lds_floats(rmax));
    if (lds < sizeof(double) * NT) lds = sizeof(double) * NT;
    if (cls == 0)
        return launch_range<4, 16>(in_dtype, epi, img, h, w, pitch, batch, taps, L, io, blocks,
                                   lds, s);
    if (cls == 1)
        return launch_range<20, 40>(in_dtype, epi, img, h, w, pitch, batch, taps, L, io, blocks,
                                    lds, s);
    return launch_range<44, 64>(in_dtype, epi, img, h, w, pitch, batch, taps, L, io, blocks, lds,
                                s);
}

}  // namespace mhfd

// ---------------------------------------------------------------------------
// Persistent form for a batch of tiles of different sizes.  Workgroups pull
// items (scale j of the class, tile, strip, segment) from a counter; items
// are numbered scale-major, so every tile's largest radius goes first.
namespace mhfd {

namespace {

template <int RLO, int RHI, typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void log_batch_kernel(int n_tiles, const BatchTile* __restrict__ tiles, int K,
                      float* __restrict__ stack, const float* __restrict__ taps, BatchScales sc,
                      BatchCounters* __restrict__ ctr, int cls) {
    extern __shared__ __attribute__((aligned(16))) float smem[];
    __shared__ int item_s;
    const int per_scale = ctr->items_per_scale;
    const int total = ctr->valid ? per_scale * sc.n : 0;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&ctr->work[cls], 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= total) break;
        const int j = item / per_scale;
        const int rem = item - j * per_scale;
        // tile: last t with item_base <= rem
        int lo = 0, hi = n_tiles;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tiles[mid].item_base <= rem)
                lo = mid;
            else
                hi = mid;
        }
        const BatchTile& t = tiles[lo];
        const int local = rem - t.item_base;
        const int strip = local % t.strips;
        const int seg = local / t.strips;
        const int x0 = strip * TW;
        const int ys = seg * t.seg_rows;
        const int ye = min(ys + t.seg_rows, t.h);
        float* out = stack + t.stack_off + static_cast<long long>(sc.plane[j]) * t.h * t.w;
        const T* img = static_cast<const T*>(t.img);
        const float* tp = taps + sc.tap_off[j];
        switch (sc.radius[j]) {
#define MHFD_BODY(R)                                                                        \
    case R:                                                                                 \
        if constexpr (R >= RLO && R <= RHI)                                                 \
            log_strip_body<R, EPI_STORE, T>(smem, img, t.h, t.w, t.pitch, tp, out, t.w, x0, \
                                            ys, ye, 0.0f, 0.0f, nullptr);                   \
        break;
            MHFD_BODY(4)
            MHFD_BODY(8)
            MHFD_BODY(12)
            MHFD_BODY(16)
            MHFD_BODY(20)
            MHFD_BODY(24)
            MHFD_BODY(28)
            MHFD_BODY(32)
            MHFD_BODY(36)
            MHFD_BODY(40)
            MHFD_BODY(44)
            MHFD_BODY(48)
            MHFD_BODY(52)
            MHFD_BODY(56)
            MHFD_BODY(60)
            MHFD_BODY(64)
#undef MHFD_BODY
            default:
                break;
        }
        __syncthreads();  // LDS is reused by the next item
    }
    (void)K;
}

template <int RLO, int RHI, typename T>
hipError_t launch_batch_typed(int n_tiles, const BatchTile* tiles, int K, float* stack,
                              const float* taps, const BatchScales& sc, BatchCounters* ctr,
                              int cls, int grid, size_t lds, hipStream_t s) {
    auto k = log_batch_kernel<RLO, RHI, T>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    k<<<grid, NT, lds, s>>>(n_tiles, tiles, K, stack, taps, sc, ctr, cls);
    return hipGetLastError();
}

template <int RLO, int RHI>
hipError_t launch_batch_range(int in_dtype, int n_tiles, const BatchTile* tiles, int K,
                              float* stack, const float* taps, const BatchScales& sc,
                              BatchCounters* ctr, int cls, int grid, size_t lds, hipStream_t s) {
    if (in_dtype == MHFD_U8)
        return launch_batch_typed<RLO, RHI, uint8_t>(n_tiles, tiles, K, stack, taps, sc, ctr, cls,
                                                     grid, lds, s);
    return launch_batch_typed<RLO, RHI, float>(n_tiles, tiles, K, stack, taps, sc, ctr, cls, grid,
                                               lds, s);
}

}  // namespace

hipError_t launch_log_batch(int cls, int in_dtype, int n_tiles, const BatchTile* tiles, int K,
                            float* stack, const float* taps, const BatchScales& sc,
                            BatchCounters* ctr, int grid, hipStream_t s) {
    if (sc.n == 0) return hipSuccess;
    int rmax = 0;
    for (int i = 0; i < sc.n; ++i) rmax = sc.radius[i] > rmax ? sc.radius[i] : rmax;
    const size_t lds = sizeof(float) * static_cast<size_t>(lds_floats(rmax));
    if (cls == 0)
        return launch_batch_range<4, 16>(in_dtype, n_tiles, tiles, K, stack, taps, sc, ctr, cls,
                                         grid, lds, s);
    if (cls == 1)
        return launch_batch_range<20, 40>(in_dtype, n_tiles, tiles, K, stack, taps, sc, ctr, cls,
                                          grid, lds, s);
    return launch_batch_range<44, 64>(in_dtype, n_tiles, tiles, K, stack, taps, sc, ctr, cls,
                                      grid, lds, s);
}

}  // namespace mhfd
