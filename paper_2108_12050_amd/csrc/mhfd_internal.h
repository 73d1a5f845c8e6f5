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

// One scale inside a LoG stack launch.
struct StackScale {
    int radius;       // padded radius (multiple of 4)
    int tap_off;      // float offset of the scale's tap block
    int plane;        // output plane index k
    int block_begin;  // first workgroup of the scale in the launch
    int n_blocks;     // strips * segments
    int seg_rows;     // rows per workgroup segment (multiple of log_chunk_rows())
};

// All scales of one radius class, in launch order (largest radius first).
struct StackLaunch {
    int n;
    int strips;       // strips of log_strip_width() columns
    int pad0, pad1;
    StackScale sc[MHFD_MAX_SCALES];
};

// Radius class of a padded radius: 0 (<= 16), 1 (<= 40), 2 (<= 64).
int log_radius_class(int padded);
int log_strip_width();
int log_chunk_rows();

// Where a stack launch writes.  Plane k of image b is at
// out + b * out_batch + k * plane_stride (row pitch = image width).
enum { EPI_STORE = 0, EPI_ACCUM = 1, EPI_SOFTSUM = 2, EPI_COTAN = 3, EPI_DUAL = 4 };
struct StackIO {
    long long img_batch;     // elements between consecutive images of a batch
    float* out;              // EPI_STORE: out = R; EPI_ACCUM: out += R
    long long out_batch;     // elements between the outputs of consecutive images
    long long plane_stride;  // elements between output planes
    double* partial;         // EPI_SOFTSUM: partial[b * total_blocks + block] =
                             //   sum of softplus(beta (|R| - tau)) over the block
    int total_blocks;        // workgroups per image in the launch
    float beta, tau;
};

// Enqueue the scale-space operator of every scale in L (all of radius class
// `cls`) for `batch` images: R = hcol (*)_y (grow (*)_x I) + gcol (*)_y (hrow
// (*)_x I) with the four tap runs at taps + sc.tap_off, and the epilogue
// `epi` (EPI_*).  u8 images support EPI_STORE only.
hipError_t launch_log_class(int cls, int in_dtype, int epi, const void* img, int h, int w,
                            int64_t pitch, int batch, const float* taps, const StackLaunch& L,
                            const StackIO& io, hipStream_t s);

// ---------------------------------------------------------------------------
// Scale-space operator on the matrix cores (split-FP16 MFMA), u8 or fp32 tiles.
// Window geometry of one radius: the row pass reads columns x0 - rw8 ...
// (nkr K-blocks of 32), the column pass rows y0 - rwc ... (nkc K-blocks).
// Shapes are (n, n), n = 1..4, for radii 0..56.
struct MfmaShape {
    int rw8, rwc, nkr, nkc;
};
constexpr int MFMA_SHAPES = 4;  // (nkr, nkc) instantiations: (1,1) ... (4,4)
constexpr int MFMA_WAVE_COLS = 16;  // image columns per matrix-core wave
constexpr int MFMA_GROUP_WAVES = 4;  // waves (adjacent wave columns) per matrix-core workgroup
bool mfma_radius_ok(int radius);
MfmaShape mfma_shape(int radius);
// FP16 fragment table of one scale: (nkr + nkc) * 4 * 64 lanes * 8 halves.
size_t mfma_frag_halves(int radius);
// Builds the table from the one-sided taps g[0..R], h[0..R] (double), the
// normalisation norm = s sigma^2, the input code scale (intensity = code /
// in_scale) and the largest code; returns the exact power-of-two output scale.
float mfma_build_frags(const double* g, const double* h, int R, double norm, double in_scale,
                       double in_max, uint16_t* dst);
int mfma_wave_tiles(int w);        // matrix-core waves across a row (MFMA_WAVE_COLS each)
int mfma_waves_per_block();

struct MfmaScale {
    int rw8, rwc;
    int frag_off;     // first 8-half fragment of the scale in the table
    int plane;        // output plane index
    int block_begin;  // first workgroup of the scale in the launch
    int n_blocks;     // groups_x * segments
    int seg_rows;     // rows per wave segment (multiple of 16)
    float out_scale;  // exact power of two
    int dev_scale_idx;  // MfmaLaunch::dev_scale: index of the scale's output factor
    // EPI_DUAL: a second column-tap set on the same row pass (same row
    // taps), its table and output factor
    int frag_off2;
    int dev_scale_idx2;
};

// Scales sharing one (nkr, nkc) instantiation.
struct MfmaLaunch {
    int n;
    int tiles_x;      // waves across a row (mfma_wave_tiles)
    int groups_x;     // workgroups across a row: ceil(tiles_x / waves per block)
    int pad;
    MfmaScale sc[MHFD_MAX_SCALES];
    // Batched fp32 launches (launch_log_mfma_soft; zero elsewhere): images
    // img_stride elements apart, outputs out_stride apart; non-null
    // dev_scale: output factors on the device (fragments built there);
    // EPI_SOFTSUM: one double per wave and image at partial, softplus of
    // beta (|R| - tau).
    long long img_stride, out_stride;
    const float* dev_scale;
    double* partial;
    float beta, tau;
    // EPI_COTAN (the soft score's backward, on the last sigma-derivative
    // term): with d = out + R and r = aux at each pixel, the cotangent
    // c = w sigma^2, w = gbar[b] inv_khw beta sigmoid(beta (|r| - tau)) sgn r,
    // replaces r in aux; the wave's sum of w (2 r / sigma + sigma^2 d) goes
    // to partial and max |c| of image b to cmax[b] (float bits).
    // EPI_DUAL: the second column set's output, plane stride 0, images
    // out_stride apart
    float* aux;
    const float* sigmas;
    int soft_k;
    const float* gbar;
    double inv_khw;
    uint32_t* cmax;
};

// Threshold-sparse stack output (mask null: the dense stack): only the
// 4-pixel row groups holding a value above tau are written; activity word
// [k][by][bx] (by < ceil(h/16), bx < ceil(w/16)) marks them, bit 16 g + r
// for row 16 by + r, columns 16 bx + 4 g ... + 3.
struct ActOut {
    uint64_t* mask;
    int bx, by;
    float tau;
};

// in_dtype MHFD_U8 or MHFD_F32.  maxbits: fp32 inputs, the float bits of the
// tile's max |I| (launch_absmax), which picks the exact input scale;
// stretched u8 inputs (stretch = 1), the levels {low, high}
// (launch_stretch_levels); otherwise unused.
hipError_t launch_log_mfma(int in_dtype, int stretch, int nkr, int nkc, const void* img, int h,
                           int w, int64_t pitch, const uint32_t* maxbits, const uint16_t* frags,
                           const MfmaLaunch& L, float* out, long long plane_stride,
                           const ActOut& act, hipStream_t s);
// The paper's DoG criterion: M = max_i sig_i (L_{i+1} - L_i) over K Gaussian
// planes and its first argmax (u8); then the blob records' k and sigma from
// the argmax plane (after the detection tail ran on M).
hipError_t launch_dog(const float* L, int K, const float* sigmas_dev, int h, int w, float* M,
                      uint8_t* arg, hipStream_t s);
hipError_t launch_dog_label(mhfd_blob* blobs, int capacity, const mhfd_result* result,
                            const uint8_t* arg, int w, const float* sigmas_dev, hipStream_t s);
// Histogram stretch of an 8-bit image: the counts go to n_copies global
// histograms copies[n_copies][256] (zeroed first, 1 <= n_copies <=
// STRETCH_MAX_COPIES), then levels[0] = low, levels[1] = high and, when hist
// is not null, hist[256] = the summed counts (hist may not alias copies).
constexpr int STRETCH_COPIES = 8;
constexpr int STRETCH_MAX_COPIES = 64;
hipError_t launch_stretch_levels(const uint8_t* img, int h, int w, long long pitch,
                                 int32_t* copies, int n_copies, int32_t* hist, int32_t* levels,
                                 int n_cu, hipStream_t s);
// *bits = float bits of max |I| over an fp32 image (zeroed first).
hipError_t launch_absmax(const float* img, int h, int w, int64_t pitch, uint32_t* bits,
                         hipStream_t s);
// max |I| word of each of `batch` dense h x w fp32 images
hipError_t launch_absmax_images(const float* imgs, int batch, int h, int w, uint32_t* bits,
                                hipStream_t s);
// The matrix-core operator over a batch of dense fp32 images (gridDim.y =
// batch) with epilogue epi (EPI_STORE / EPI_ACCUM into out, plane stride 0,
// EPI_SOFTSUM into L.partial, EPI_COTAN as MfmaLaunch describes, EPI_DUAL:
// the first column set into out and the second into L.aux); maxbits[b]:
// max |I| word of image b.
hipError_t launch_log_mfma_soft(int epi, int nkr, int nkc, const float* img, int h, int w,
                                int batch, const uint32_t* maxbits, const uint16_t* frags,
                                const MfmaLaunch& L, float* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Frequency-domain scale-space operator (plan mode MHFD_BLUR_FFT), fft_blur.hip.
constexpr int FFT_MAX_N = MHFD_MAX_FFT_SIZE;  // longest transform (power of two)
struct FftTables {      // device pointers, owned by the plan
    const float* lam;       // [k][g, h][nmax] spectral weights at nmax
    const float2* tw;       // e^{-2 pi i k / nmax}, k < nmax
    const float2* q;        // e^{-i pi k / (2 nmax)}, k < nmax
    int K;
    int nmax;
    float norm[MHFD_MAX_SCALES];  // s sigma_k^2 (host copy)
};
bool fft_size_ok(int n);
// floats of scratch per call for an h x w tile
size_t fft_workspace_floats(int h, int w);
// Spectral weights of every scale (one-sided double taps g_0..g_R, h_0..h_R
// per scale at taps + tap_off[k]) into lam, once per plan.
hipError_t build_fft_spectra(const double* taps, const int* tap_off, const int* radii, int K,
                             int nmax, float* lam, hipStream_t s);
hipError_t launch_fft_log_stack(const FftTables& T, int in_dtype, const void* img, int h, int w,
                                int64_t pitch, float* stack, float* ws, hipStream_t s);

// Detection tail: stack -> candidates -> canonical order -> prune -> blobs.
struct DetectWorkspace {
    const float* stack;      // K x h x w
    int32_t* blk_n;          // per NMS block: candidate count
    int32_t* blk_o;          // per NMS block: offset in the pool
    int32_t* blk_off;        // per NMS block: exclusive scan of blk_n (n_blk + 1)
    Cand* pool;              // unordered records: per-workgroup slots, then overflow
    Cand* cand;              // candidates in canonical order
    int32_t* keep;           // keep flag per candidate
    int32_t* keep_off;       // exclusive scan of keep (cap + 1)
    int32_t* scan_sums;      // span sums of the scans (scan_sums_ints of the longer input)
    DetectCounters* ctr;
    int64_t cap;             // candidate capacity
    int n_blk;               // number of NMS blocks
    int blk_per_row;         // NMS blocks per image row
    // Threshold-sparse stack (null: dense): K x act_by x act_bx words, bit
    // 16 g + r of word [k][by][bx] set when row 16 by + r, columns 16 bx +
    // 4 g ... + 3 of plane k hold a value above the threshold and were
    // written; other groups of the stack are not read.
    const uint64_t* act = nullptr;
    int act_bx = 0, act_by = 0;
};

// d2max: K x K table, d2max[ka * K + kb] = largest squared integer distance at
// which blobs of scales ka and kb overlap by more than the plan's threshold
// (-1: never); null disables pruning.  `d2top` = max d2max, `reach` =
// floor(sqrt(d2top)).
hipError_t launch_detect_tail(const DetectWorkspace& ws, int K, int h, int w, float tau,
                              const int32_t* d2max, int reach, int d2top, const float* sigmas_dev,
                              mhfd_blob* blobs, int capacity, mhfd_result* result, hipStream_t s);

// Records of the unordered candidate pool: a fixed slot per NMS workgroup
// plus a shared overflow region of `cap` records.
size_t nms_pool_records(int n_blk, int64_t cap);

// Ints of span-sum scratch a scan over n items needs.
size_t scan_sums_ints(int64_t n);

int nms_blocks_per_row(int w);

// Workgroups per row offset of the prune launches (grid rows = 2 reach + 1):
// about 4096 workgroups in all.
inline int prune_grid_x(int span) { return span >= 4096 ? 1 : (4096 + span - 1) / span; }

// ---------------------------------------------------------------------------
// Batched detection.  The setup kernel turns the caller's device descriptors
// into this per-tile table and the work prefixes below.
struct BatchTile {
    const void* img;
    long long pitch;
    long long stack_off;    // first float of the tile's K planes in the stack
    mhfd_blob* blobs;
    mhfd_result* result;
    int h, w;
    int capacity;
    int seg_rows;
    int strips, segs;       // LoG workgroups per scale: strips * segs
    int bpr;                // maxima cells per row (strips of 64 nms_cw columns)
    int item_base;          // prefix of strips * segs over earlier tiles
    int nms_base;           // prefix of h * bpr over earlier tiles
    int nms_cw;             // columns per maxima lane (1, 2 or 4)
    int nitem_base;         // prefix of ceil(h / 32) * bpr (maxima wave items)
    // matrix-core items: workgroups of MFMA_GROUP_WAVES wave columns x row
    // segments
    int mtiles_x, msegs, mseg_rows;
    int mgroups_x;          // ceil(mtiles_x / MFMA_GROUP_WAVES)
    int mitem_base;         // prefix of mgroups_x * msegs over earlier tiles
    long long act_off;      // first activity word of the tile (threshold-sparse stack):
                            // K x ceil(h/16) x ceil(w/16) words
};

// Activity words a batch may need: K x sum over tiles of ceil(h/16) ceil(w/16)
// <= K (max_pixels / 256 + n ((max_h + max_w) / 16 + 1)).
inline long long batch_act_words(int K, int n, long long max_pixels, int max_h, int max_w) {
    return static_cast<long long>(K) *
           (max_pixels / 256 + static_cast<long long>(n) * ((max_h + max_w) / 16 + 2));
}

struct BatchCounters {
    int32_t items_per_scale;  // sum over tiles of strips * segs
    int32_t nms_blocks;       // sum over tiles of h * bpr (maxima cells)
    int32_t nms_items;        // sum over tiles of ceil(h / 16) * bpr (maxima waves)
    int32_t valid;            // 1 when every descriptor passed the checks
    int32_t pool_used;
    int32_t flags;
    int32_t n_cand;
    int32_t n_blobs;
    int32_t work[3];          // persistent LoG work counters, one per radius class
    int32_t mitems_per_scale; // sum over tiles of mgroups_x * msegs (workgroup items)
    int32_t mwork[MFMA_SHAPES];  // persistent matrix-core work counters, one per shape
};

// Scales of one (nkr, nkc) shape for the persistent matrix-core launch.
struct MfmaBatchScales {
    int n;
    int rw8[MHFD_MAX_SCALES], rwc[MHFD_MAX_SCALES];
    int frag_off[MHFD_MAX_SCALES], plane[MHFD_MAX_SCALES];
    float out_scale[MHFD_MAX_SCALES];
};

// act: the batch's activity words (null: dense stacks), tau the threshold.
hipError_t launch_log_mfma_batch(int in_dtype, int nkr, int nkc, int n_tiles,
                                 const BatchTile* tiles, const uint32_t* maxbits, float* stack,
                                 const uint16_t* frags, const MfmaBatchScales& sc,
                                 BatchCounters* ctr, int slot, int grid, uint64_t* act, float tau,
                                 hipStream_t s);
// bits[t] = float bits of max |I| of fp32 tile t (zeroed first; nothing for an
// invalid batch).
hipError_t launch_absmax_batch(int n_tiles, const BatchTile* tiles, const BatchCounters* ctr,
                               uint32_t* bits, int grid, hipStream_t s);

// Scales of one radius class for the persistent LoG launch.
struct BatchScales {
    int n;
    int radius[MHFD_MAX_SCALES];
    int tap_off[MHFD_MAX_SCALES];
    int plane[MHFD_MAX_SCALES];
};

hipError_t launch_log_batch(int cls, int in_dtype, int n_tiles, const BatchTile* tiles,
                            int K, float* stack, const float* taps, const BatchScales& sc,
                            BatchCounters* ctr, int grid, hipStream_t s);

struct BatchLaunchArgs {
    int K, n_tiles, n_blk_bound, nms_grid, reach, d2top;
    float tau;
    int64_t cap;
    const float* stack;
    const uint64_t* act;    // threshold-sparse stacks' activity words (null: dense)
    const BatchTile* tiles;
    int32_t *blk_n, *blk_o, *blk_off, *keep, *keep_off, *scan_sums;
    Cand *pool, *cand;
    const int32_t* d2max;   // null: no pruning
    const float* sigmas;
    BatchCounters* ctr;
};

// mfma: the plan computes some scales on the matrix cores, so the
// setup also numbers the matrix-core items.
hipError_t launch_batch_setup(const mhfd_tile* in, int n, long long max_pixels, int K, int max_h,
                              int max_w, int dtype, int mfma, BatchTile* tiles,
                              BatchCounters* ctr, hipStream_t s);

hipError_t launch_batch_tail(const BatchLaunchArgs& a, hipStream_t s);

// Exclusive scan of n = min(n_host, *n_dev) ints (n_dev may be null):
// out[0..n], total also to *total_out when given.  `sums` needs
// scan_sums_ints(n_host) ints.
void launch_batch_scan(const int32_t* in, int n_host, const int32_t* n_dev, int32_t* sums,
                       int32_t* out, int32_t* total_out, hipStream_t s);

// Device-synthesised taps of the soft focus score: for scale k, four tap sets
// (FWD, D1, D2, ADJ) of four runs of padded[k] + 1 floats start at offset[k].
// The radius of scale k, floor(truncate sigma_k + 0.5), comes from the
// device sigma at each call; taps beyond it are zero.  padded[k] is scale
// k's launch radius: a sigma is accepted when it lies in (0, sigma_cap] and
// its radius fits the launch radius.
enum { SOFT_FWD = 0, SOFT_D1 = 1, SOFT_D2 = 2, SOFT_ADJ = 3, SOFT_SETS = 4 };
struct SoftTapLayout {
    int K;
    float truncate;
    float sigma_cap;                 // +inf: bounded by the launch radii only
    int padded[MHFD_MAX_SCALES];
    int offset[MHFD_MAX_SCALES];
};

// err (optional): 0, or MHFD_FOCUS_BAD_SIGMA when some sigma is not accepted
// (its taps are written as zeros).
hipError_t launch_soft_taps(const float* sigmas, const SoftTapLayout& lay, float* taps,
                            int32_t* err, hipStream_t s);
// Softplus partials of the forward launches: launch c wrote [image][block]
// (blocks[c] per image) starting at partial + base[c].
struct SoftPartials {
    int n;
    long long base[4];
    int blocks[4];
};
// Matrix-core form of the soft score: fragment tables of every (scale, tap
// set) built on the device from the synthesised taps, at the shape of the
// scale's launch radius; set s of scale k at frag + off[k] + s * halves[k]
// (FP16 halves), output factor at scales[4 k + s].
struct SoftFragLayout {
    int K;
    int nkr[MHFD_MAX_SCALES], nkc[MHFD_MAX_SCALES], rw8[MHFD_MAX_SCALES], rwc[MHFD_MAX_SCALES];
    long long off[MHFD_MAX_SCALES];
    int halves[MHFD_MAX_SCALES];
};
hipError_t launch_soft_frags(const float* taps, const SoftTapLayout& lay, const SoftFragLayout& fl,
                             uint16_t* frags, float* scales, hipStream_t s);
hipError_t launch_soft_finish(const double* partial, const SoftPartials& sp, int batch,
                              double inv_khw, float* scores, hipStream_t s);
// Sigma-gradient partials per scale of the cotangent pass ([image][workgroup]).
int soft_cotangent_blocks(int batch);
// r <- c = w sigma^2 (per pixel of each image), partial[] <- the sigma
// partials; cmax (optional, `batch` words): max |c| of each image.
hipError_t launch_soft_cotangent(float* r, const float* d, long long n_per_image, int batch,
                                 const float* sigmas, int k, const float* gbar, double inv_khw,
                                 float beta, float tau, double* partial, uint32_t* cmax,
                                 hipStream_t s);
// p[0 .. n) = 0 (a fill kernel, safe under graph capture)
hipError_t launch_zero_f64(double* p, long long n, hipStream_t s);
hipError_t launch_sigma_grad_finish(const double* partial, int nb, int K, float* dsig,
                                    hipStream_t s);

}  // namespace mhfd
