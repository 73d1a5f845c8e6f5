// Internal declarations shared by the libmhfd translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhfd.h"

namespace mhfd {

// Radii are rounded up to a multiple of 4 for kernel instantiation; the extra
// taps are zero, so the padded sums equal the unpadded ones exactly.
constexpr int kRadiusQuantum = 4;
constexpr int kMaxPaddedRadius = MHFD_MAX_RADIUS;

inline int padded_radius(int r) { return ((r + kRadiusQuantum - 1) / kRadiusQuantum) * kRadiusQuantum; }

// Half-sample symmetric extension of index u into [0, n).
__host__ __device__ __forceinline__ int reflect_index(int u, int n) {
    if (u >= 0 && u < n) return u;
    int p = 2 * n;
    int m = u % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

// Tap table of one scale, padded radius P: four runs of (P + 1) floats,
// index j = 0..P (taps are symmetric):
//   [0]        g_j                row-pass Gaussian
//   [P+1]      h_j                row-pass second derivative
//   [2(P+1)]   s sigma^2 g_j      column-pass Gaussian with the normalisation
//   [3(P+1)]   s sigma^2 h_j      column-pass second derivative
inline int tap_block_floats(int padded) { return 4 * (padded + 1); }

// One candidate record inside the detection workspace.
struct Cand {
    int32_t y, x, k;
    float r;
};

struct DetectCounters {
    int32_t pool_used;   // records reserved in the unordered pool
    int32_t flags;       // MHFD_FLAG_*
    int32_t n_cand;      // total candidates (after the block scan)
    int32_t n_blobs;     // total blobs after pruning
};

// Launch the LoG strip kernel for one scale: writes R_k (h x w, pitch
// out_pitch) from the image.  `padded` selects the instantiation.
hipError_t launch_log_scale(int padded, int in_dtype, const void* img, int h, int w, int64_t pitch,
                            const float* taps, float* out, int64_t out_pitch, int seg_rows,
                            hipStream_t s);

// Detection tail: stack -> candidates -> canonical order -> prune -> blobs.
struct DetectWorkspace {
    const float* stack;      // K x h x w
    int32_t* blk_n;          // per NMS block: candidate count
    int32_t* blk_o;          // per NMS block: offset in the pool
    int32_t* blk_off;        // per NMS block: exclusive scan of blk_n (n_blk + 1)
    Cand* pool;              // unordered candidate records
    Cand* cand;              // candidates in canonical order
    int32_t* keep;           // keep flag per candidate
    int32_t* keep_off;       // exclusive scan of keep (cap + 1)
    DetectCounters* ctr;
    int64_t cap;             // candidate capacity
    int n_blk;               // number of NMS blocks
    int blk_per_row;         // NMS blocks per image row
};

// `reach`: rows farther apart than this cannot hold overlapping blobs
// (floor(2 sqrt(2) sigma_max)).
hipError_t launch_detect_tail(const DetectWorkspace& ws, int K, int h, int w, float tau,
                              float overlap, int reach, const float* sigmas_dev, mhfd_blob* blobs,
                              int capacity, mhfd_result* result, hipStream_t s);

int nms_blocks_per_row(int w);

}  // namespace mhfd
