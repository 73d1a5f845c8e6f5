/*
 * mhfd.h -- C ABI of libmhfd: the scale-normalised Laplacian-of-Gaussian
 * (LoG) blob detector used as a focus criterion for serial-section electron
 * microscopy ("Ultrafast Focus Detection for Automated Microscopy",
 * Multi-scale Histologic Feature Detection), written in HIP for AMD MI355X
 * (gfx950).
 *
 * What the library computes, for an image I and scales sigma_1 < ... < sigma_K
 * (section 2.2: Gaussian G, scale space L = G_t * I with t the standard
 * deviation, scale grid t_i = min_t + (i-1) delta_t):
 *
 *   R_k(y,x)  = s * sigma_k^2 * Lap(G_sigma_k * I)(y,x)        the stack
 *     sampled Gaussian taps g over |j| <= floor(truncate*sigma + 0.5),
 *     normalised to unit sum; second-derivative taps h_j = (j^2 - V) g_j /
 *     sigma^4 with V the variance of the truncated kernel (zero sum); borders
 *     extended half-sample symmetrically (... x1 x0 | x0 x1 ...); s = -1 for
 *     bright blobs (default), +1 for dark.  This is the scale-normalised
 *     Laplacian t^2 Lap L that section 2.2 approximates by a difference of
 *     Gaussians.
 *   candidates: voxels (y, x, k) equal to the maximum of their 3x3x3
 *     scale-space window (windows clipped at the volume's faces) with
 *     R_k(y,x) > threshold -- the maxpool-equality test of section 3
 *     (equation "argmax"), taken local in scale as well as in space;
 *   pruning: a candidate b is dropped when some other candidate a dominates
 *     it (larger k, or equal k and smaller (y, x)) and the discs of radius
 *     sqrt(2)*sigma around them overlap by more than `overlap` of the
 *     smaller disc's area (one-shot rule, FP64 geometry);
 *   focus criterion: the number of surviving blobs, |C| (section 3,
 *     Algorithm 1's output); its density per megapixel compares tiles of
 *     different sizes.
 *
 * Soft focus score (differentiable form):
 *   S_b = 1/(K H W) sum_k sum_{y,x} softplus(beta * (|r_k(y,x)| - tau)),
 *   r_k = sigma_k^2 Lap(G_sigma_k * I_b), with its gradient with respect to
 *   every image and every sigma.
 *
 * Conventions shared by every call:
 *   - All pointers named d_* are device pointers on the device that was
 *     current when the plan was created; the caller owns and allocates them.
 *     Host pointers are named without the prefix.
 *   - Images are row-major; `pitch` is the distance between rows in elements
 *     (>= w).  Float images hold any finite values; 8-bit images are read as
 *     u / 255.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call that
 *     takes a stream only enqueues work on it and returns without waiting;
 *     results are valid once the stream has reached that point.
 *   - Argument and size errors are found on the host before anything is
 *     enqueued and reported as a status; nothing is written then.  A failing
 *     HIP call gives MHFD_ERR_HIP.  mhfd_last_error() returns a description
 *     of the last failure on the calling thread.
 *   - Calls on one plan may run concurrently on different streams as long as
 *     they use different workspaces and outputs; a plan is read-only after
 *     creation.
 */
#ifndef MHFD_H
#define MHFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHFD_MAX_SCALES 32   /* largest K */
#define MHFD_MAX_RADIUS 64   /* largest kernel radius floor(truncate*sigma + 0.5) */
#define MHFD_MAX_BATCH 4096  /* largest number of tiles in one batched call */

typedef enum mhfd_status {
    MHFD_OK = 0,
    MHFD_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad configuration */
    MHFD_ERR_UNSUPPORTED = 2, /* valid request outside what this build supports */
    MHFD_ERR_WORKSPACE = 3,   /* workspace smaller than the size query returned */
    MHFD_ERR_HIP = 4,         /* a HIP runtime call failed */
    MHFD_ERR_OOM = 5          /* device allocation for the plan failed */
} mhfd_status;

typedef enum mhfd_dtype { MHFD_F32 = 0, MHFD_U8 = 1 } mhfd_dtype;
typedef enum mhfd_polarity { MHFD_BRIGHT = 0, MHFD_DARK = 1 } mhfd_polarity;

/* One detected blob (20 bytes).  Lists are in ascending (y, x, k) order. */
typedef struct mhfd_blob {
    int32_t y, x;      /* pixel position */
    int32_t k;         /* scale index, 0-based */
    float sigma;       /* sigma_k */
    float response;    /* R_k(y, x) */
} mhfd_blob;

/* Summary of one detection, written by the device (32 bytes). */
typedef struct mhfd_result {
    int64_t n_blobs;       /* blobs after pruning: the focus criterion |C| */
    int64_t n_candidates;  /* window maxima above the threshold, before pruning */
    int32_t flags;         /* MHFD_FLAG_* */
    int32_t reserved;
    double density;        /* n_blobs per megapixel, n_blobs * 1e6 / (h w): the
                              criterion for tiles of different sizes */
} mhfd_result;

/* n_blobs exceeds the caller's capacity: only the first `capacity` blobs of
 * the canonical order were written (n_blobs is still the true count). */
#define MHFD_FLAG_BLOB_OVERFLOW 1
/* n_candidates exceeds the plan's max_candidates: pruning could not see every
 * candidate and n_blobs and the list are not valid. */
#define MHFD_FLAG_CAND_OVERFLOW 2

/*
 * Detection criterion of a plan.
 *   LOG  the scale-normalised LoG stack and its 3x3x3 window maxima above
 *        the threshold, then overlap pruning (the default: the exact
 *        Laplacian that the DoG approximates, with local maxima in scale).
 *   DOG  the paper's own criterion (equation "dog" of section 2.2,
 *        equation "argmax" and Algorithm 1 of section 3): Gaussian
 *        planes L_k at the K scales; DoG_i = t_i (L_{i+1} - L_i) for
 *        i < K - 1; per pixel the largest DoG over scale and its first
 *        argmax i; a blob at every pixel whose
 *        largest DoG exceeds the threshold and equals the maximum of its
 *        3x3 neighbourhood (clipped at the border).  Records carry k = that
 *        argmax and sigma_k.  Needs K >= 2, every radius <= 56 (matrix-core
 *        path) and overlap >= 1 (no pruning); the stack of mhfd_log_stack /
 *        mhfd_detect (d_stack) then holds the Gaussian planes L_k.  The sign
 *        is the paper's: dark blobs on a bright background respond
 *        positively (the polarity field is ignored).
 */
#define MHFD_CRITERION_LOG 0
#define MHFD_CRITERION_DOG 1

/*
 * How a plan computes the stack (the convolution of section 3).
 *   DIRECT  separable convolution on the matrix cores (radius <= 56) or the
 *           vector units (radius <= MHFD_MAX_RADIUS); cost grows with sigma.
 *   FFT     products of transforms: the image's 2-D DCT-II (the Fourier
 *           transform of its half-sample symmetric extension) times each
 *           scale's kernel spectrum, then the inverse DCT; cost independent
 *           of sigma, radius up to MHFD_MAX_FFT_RADIUS.  Images must have
 *           power-of-two sides of at most MHFD_MAX_FFT_SIZE
 *           (MHFD_ERR_UNSUPPORTED otherwise); the LoG criterion only, no
 *           stretch; detection only (batched and focus-score calls refuse
 *           such plans; no threshold-sparse stack).  FP32 arithmetic,
 *           twiddles and spectra built in FP64 (the spectra once per plan,
 *           on the device, at the plan's largest power-of-two side).
 *           Measured error against the FP64 direct convolution: about 3e-7
 *           of each plane's maximum.
 */
#define MHFD_BLUR_DIRECT 0
#define MHFD_BLUR_FFT 1
#define MHFD_MAX_FFT_SIZE 4096
#define MHFD_MAX_FFT_RADIUS 2048

typedef struct mhfd_config {
    int32_t n_scales;        /* K, 1..MHFD_MAX_SCALES */
    float sigma_min;         /* linear grid sigma_k = min + k (max - min)/(K - 1), */
    float sigma_max;         /*   computed in double and rounded to float       */
    const float *sigmas;     /* optional host array of K strictly increasing
                                positive sigmas; overrides min/max when set    */
    float truncate;          /* kernel radius floor(truncate * sigma + 0.5); 4  */
    float threshold;         /* candidate iff R > threshold                     */
    float overlap;           /* pruning threshold in [0, 1]; >= 1 disables it   */
    int32_t polarity;        /* mhfd_polarity                                   */
    int32_t in_dtype;        /* mhfd_dtype of the images given to detect        */
    int32_t max_h, max_w;    /* largest image the plan will see                 */
    int64_t max_candidates;  /* candidate capacity of a detection workspace
                                (0: max(65536, max_h*max_w/64))                 */
    int32_t stretch;         /* 1: histogram-stretch every image first (section
                                4, Algorithm 1's first step; see
                                mhfd_stretch_levels).  8-bit plans whose radii
                                all take the matrix-core path (<= 56) only;
                                batched and focus-score calls refuse such a
                                plan (MHFD_ERR_UNSUPPORTED).  0: no stretch    */
    int32_t criterion;       /* MHFD_CRITERION_LOG (0) or MHFD_CRITERION_DOG (1) */
    float sigma_cap;         /* focus-score calls (trainable scales): > 0, the
                                largest sigma any scale may be given; its
                                radius floor(truncate * sigma_cap + 0.5) <=
                                MHFD_MAX_RADIUS sizes the halos of every scale
                                (>= every sigma of the plan).  0: each scale's
                                halo is its plan radius rounded up to a
                                multiple of 4, and a sigma may move while its
                                radius stays within that                       */
    int32_t blur;            /* MHFD_BLUR_DIRECT (0) or MHFD_BLUR_FFT (1)       */
} mhfd_config;

typedef struct mhfd_plan_s *mhfd_plan;

/* Build a plan: validates the configuration, derives every scale's kernel
 * radius and taps in double precision on the host and copies the float taps
 * to the current device (a few kilobytes, owned by the plan).  *out is set
 * only on success.  Host call; synchronous. */
mhfd_status mhfd_create_plan(const mhfd_config *cfg, mhfd_plan *out);

/* Release the plan and its device table.  The caller must make sure no
 * enqueued work still uses it.  NULL is accepted. */
mhfd_status mhfd_destroy_plan(mhfd_plan plan);

/* Read back the plan's scales (sigmas[K]) and radii (radii[K]); either
 * pointer may be NULL.  Returns K, or -1 for a NULL plan. */
int32_t mhfd_plan_scales(mhfd_plan plan, float *sigmas, int32_t *radii);

/* Workspace bytes mhfd_detect needs for an h x w image (0 on bad input). */
size_t mhfd_detect_workspace_size(mhfd_plan plan, int32_t h, int32_t w);

/*
 * Detect blobs in one image (section 3's criterion with the readings above).
 *   d_img     h x w image of the plan's dtype, row pitch `pitch` elements.
 *   d_blobs   room for `capacity` (>= 0) blobs; the first
 *             min(n_blobs, capacity) are written in ascending (y, x, k).
 *   d_result  one mhfd_result, always written.
 *   d_stack   optional K x h x w float array (plane k at k*h*w) that receives
 *             the whole LoG stack R; with NULL the detector keeps only the
 *             part above the threshold, in the workspace (threshold-sparse,
 *             see mhfd_log_stack_sparse), when the plan allows it.
 *   d_ws      workspace of at least mhfd_detect_workspace_size(plan, h, w)
 *             bytes, 256-byte aligned; its contents need no initialisation
 *             and are scratch after the call.
 * Requires 1 <= h <= max_h, 1 <= w <= max_w, pitch >= w.
 */
mhfd_status mhfd_detect(mhfd_plan plan, const void *d_img, int32_t h, int32_t w, int64_t pitch,
                        mhfd_blob *d_blobs, int32_t capacity, mhfd_result *d_result,
                        float *d_stack, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Bytes of device scratch mhfd_log_stack needs for an h x w image (0 on bad
 * input, and for 8-bit plans without the stretch, which need none).  fp32
 * plans keep one word: the image's max |I|, from which the matrix-core
 * kernels take an exact power-of-two input scale.  Stretch plans keep eight
 * copies of the 256-bin histogram and the two levels (2050 words).  FFT plans
 * keep three h x w float transform buffers.
 */
size_t mhfd_log_stack_workspace_size(mhfd_plan plan, int32_t h, int32_t w);

/*
 * The LoG stack alone -- the first step of mhfd_detect: writes
 * R_k(y, x) for k < K into d_stack (K x h x w floats, plane k at k*h*w).
 * Same image requirements as mhfd_detect.  d_ws: at least
 * mhfd_log_stack_workspace_size bytes of caller-owned device memory, 4-byte
 * aligned (may be null when that size is 0); the call overwrites it, so calls
 * in flight at once need separate workspaces.  fp32 images with non-finite
 * values give unspecified stacks.
 */
mhfd_status mhfd_log_stack(mhfd_plan plan, const void *d_img, int32_t h, int32_t w, int64_t pitch,
                           float *d_stack, void *d_ws, size_t ws_bytes, void *stream);

/*
 * mhfd_log_stack without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The call's scratch (the fp32 range word,
 * or the stretch histogram copies and levels, 8200 bytes: at most
 * MHFD_STATIC_SCRATCH_BYTES) is
 * a static array of the library, one per device, kept until the process
 * ends; the call allocates nothing.  Every call on a device shares that
 * array: calls that overlap in time on one device (on different streams, or
 * from several host threads) race and give wrong stacks, so serialise them;
 * each call clears what it uses.  Same arguments, results and errors as
 * mhfd_log_stack, plus MHFD_ERR_UNSUPPORTED if the plan needed more scratch
 * than the array holds.
 */
#define MHFD_STATIC_SCRATCH_BYTES 16384
mhfd_status mhfd_log_stack_static(mhfd_plan plan, const void *d_img, int32_t h, int32_t w,
                                  int64_t pitch, float *d_stack, void *stream);

/*
 * Histogram stretch levels of one 8-bit image (section 3; Algorithm 1, first
 * step: 0.175% of the pixels saturated at each end).  With N = h w and
 * q = 0.00175 N, low is the smallest code v with at least q pixels <= v and
 * high the largest code with at least q pixels >= v (compared exactly in
 * integers: 100000 count >= 175 N).  A stretch plan maps code v to
 * clip((v - low) / (high - low), 0, 1), and every code to 0 when high = low.
 *   d_img     h x w codes, row pitch `pitch` >= w bytes; h w < 2^31.
 *   d_hist    256 int32, receives the histogram (count of each code).
 *   d_levels  2 int32, receives {low, high}.
 * Device pointers, caller-owned; enqueued on `stream` (the current device's
 * compute units size the launch).  No plan and no workspace: the outputs are
 * the scratch, so every workgroup adds its counts to the one d_hist (the
 * detector's own stretch pass spreads them over eight copies in its
 * workspace, a few microseconds faster on a 4096 x 4096 tile).  Errors: MHFD_ERR_INVALID_ARG for null pointers or bad sizes,
 * MHFD_ERR_UNSUPPORTED above 2^31 - 1 pixels, MHFD_ERR_HIP for launch
 * failures; nothing is enqueued on error.
 */
mhfd_status mhfd_stretch_levels(const uint8_t *d_img, int32_t h, int32_t w, int64_t pitch,
                                int32_t *d_hist, int32_t *d_levels, void *stream);

/*
 * The rest of mhfd_detect on a stack the caller already holds (as written by
 * mhfd_log_stack): maxima, threshold, canonical list, pruning, count.
 * mhfd_log_stack followed by mhfd_detect_stack gives exactly what
 * mhfd_detect gives.  d_ws as for mhfd_detect (its stack region is unused).
 */
mhfd_status mhfd_detect_stack(mhfd_plan plan, const float *d_stack, int32_t h, int32_t w,
                              mhfd_blob *d_blobs, int32_t capacity, mhfd_result *d_result,
                              void *d_ws, size_t ws_bytes, void *stream);

/*
 * The two halves of mhfd_detect in the form it takes without a caller stack
 * (threshold-sparse).  A voxel at or below the threshold can neither be a
 * candidate nor block one (a neighbour that blocks a candidate exceeds it,
 * and so the threshold), so the detector writes and reads only the 4-pixel
 * row groups of the stack that hold a value above the threshold, and marks
 * them in activity words: word [k][by][bx] (by < ceil(h/16), bx <
 * ceil(w/16)) has bit 16 g + r set when row 16 by + r, columns 16 bx + 4 g
 * ... 16 bx + 4 g + 3 of plane k hold such a value (those four values are
 * then written; the other groups of d_stack are left as they were).
 *   mhfd_activity_bytes  bytes of the activity words for an h x w image;
 *                        0 for plans without this form (the DoG criterion,
 *                        a radius above 56, or a negative threshold) and on
 *                        bad input.
 *   mhfd_log_stack_sparse   as mhfd_log_stack, plus d_act (8-byte aligned,
 *                           mhfd_activity_bytes bytes, every word written).
 *   mhfd_detect_stack_sparse  as mhfd_detect_stack on such a stack.
 * mhfd_log_stack_sparse followed by mhfd_detect_stack_sparse gives exactly
 * what mhfd_detect gives; MHFD_ERR_UNSUPPORTED for plans without the form.
 */
size_t mhfd_activity_bytes(mhfd_plan plan, int32_t h, int32_t w);
mhfd_status mhfd_log_stack_sparse(mhfd_plan plan, const void *d_img, int32_t h, int32_t w,
                                  int64_t pitch, float *d_stack, uint64_t *d_act, void *d_ws,
                                  size_t ws_bytes, void *stream);
mhfd_status mhfd_detect_stack_sparse(mhfd_plan plan, const float *d_stack, const uint64_t *d_act,
                                     int32_t h, int32_t w, mhfd_blob *d_blobs, int32_t capacity,
                                     mhfd_result *d_result, void *d_ws, size_t ws_bytes,
                                     void *stream);

/* One image of a batch (device-resident descriptor, 48 bytes). */
typedef struct mhfd_tile {
    const void *img;       /* device image of the plan's dtype                  */
    int32_t h, w;          /* 1 <= h <= max_h, 1 <= w <= max_w                  */
    int64_t pitch;         /* row pitch in elements, >= w                       */
    mhfd_blob *blobs;      /* device: room for `capacity` blobs                 */
    mhfd_result *result;   /* device: one result, always written               */
    int32_t capacity;      /* >= 0                                              */
    int32_t seg_rows;      /* rows per LoG workgroup for this tile: 0 = library
                              default, else a multiple of 32 in [32, 4096]      */
} mhfd_tile;

/* A descriptor failed the device-side checks (or the batch exceeded the
 * workspace bounds); nothing was computed for the batch. */
#define MHFD_FLAG_INVALID_TILE 4

/* Launch shape of a batched call; NULL (or a field of 0) takes the default.
 * The results do not depend on it, only the time does (the autotuner of the
 * Python layer chooses it).
 *   log_groups_per_cu  persistent LoG workgroups per compute unit, 1..8 (2)
 *   nms_groups_per_cu  persistent maxima workgroups per compute unit, 1..32 (8)
 * Values outside the ranges give MHFD_ERR_INVALID_ARG. */
typedef struct mhfd_batch_opts {
    int32_t log_groups_per_cu;
    int32_t nms_groups_per_cu;
} mhfd_batch_opts;

/* Workspace bytes mhfd_detect_batched needs for up to max_tiles tiles with at
 * most max_pixels pixels in total (0 on bad input). */
size_t mhfd_batch_workspace_size(mhfd_plan plan, int32_t max_tiles, int64_t max_pixels);

/*
 * Detect blobs in n tiles of different sizes at once: the same results per
 * tile as mhfd_detect (bit for bit), from one fixed sequence of launches.
 *   d_tiles   n device descriptors.  The host never reads them: a setup kernel
 *             checks them on the device, so the call can be captured in a HIP
 *             graph once and replayed with new descriptors of any sizes within
 *             the bounds.  If any descriptor is invalid, or the tiles hold more
 *             than max_pixels pixels, every tile's result gets
 *             MHFD_FLAG_INVALID_TILE with zero counts and no tile is processed.
 *   max_pixels, d_ws, ws_bytes  bounds the workspace was sized for
 *             (mhfd_batch_workspace_size(plan, n_max, max_pixels), n <= n_max).
 *   opts      launch shape (mhfd_batch_opts), NULL for the defaults.
 * Scales of a radius class run as persistent workgroups that pull
 * (scale, tile, strip, segment) items, largest radius first.
 */
mhfd_status mhfd_detect_batched(mhfd_plan plan, int32_t n, const mhfd_tile *d_tiles,
                                int64_t max_pixels, const struct mhfd_batch_opts *opts,
                                void *d_ws, size_t ws_bytes, void *stream);

/* Workspace bytes mhfd_focus_score and mhfd_focus_score_backward need for a
 * batch of b images of h x w (0 on bad input). */
size_t mhfd_focus_workspace_size(mhfd_plan plan, int32_t b, int32_t h, int32_t w);

/* A sigma given to a focus-score call is outside what the plan's halos
 * allow (see mhfd_config.sigma_cap) or not finite: that call's scores and
 * gradients are not valid. */
#define MHFD_FOCUS_BAD_SIGMA 1

/*
 * Soft focus score of b float images (b x h x w, dense).
 *   d_sigmas  K device floats, the current (trainable) scales.  Each call
 *             derives every scale's taps and kernel radius
 *             floor(truncate * sigma_k + 0.5) on the device from these values
 *             (section 2.2's sampled Gaussian at the current sigma, truncated
 *             as the plan's own scales are); the score is smooth in sigma
 *             between the sigmas where a radius changes.  The halos are sized
 *             for the plan's sigma_cap.
 *   d_scores  b floats, overwritten with S_b.
 *   d_error   optional device int32 (may be NULL), overwritten with 0 or
 *             MHFD_FOCUS_BAD_SIGMA when some sigma is not positive, exceeds
 *             sigma_cap, or (sigma_cap = 0) has a radius above its halo
 *             (that scale's taps are then zero).  The host cannot see device
 *             values without waiting, so this is the call's only report of
 *             a bad sigma; read it after the stream has passed the call.
 * Requires 1 <= h <= max_h, 1 <= w <= max_w, b >= 1; beta > 0.
 */
mhfd_status mhfd_focus_score(mhfd_plan plan, const float *d_imgs, int32_t b, int32_t h, int32_t w,
                             const float *d_sigmas, float beta, float tau, float *d_scores,
                             int32_t *d_error, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Gradient of sum_b d_grad_scores[b] * S_b.
 *   d_grad_imgs    b x h x w floats, overwritten with the image gradient.
 *   d_grad_sigmas  K floats, overwritten with the sigma gradient: the
 *                  derivative at the radii of the current sigmas (the radius
 *                  is piecewise constant in sigma).
 * The stack is recomputed per scale; nothing from the forward call is kept.
 * Same arguments, requirements and d_error report as mhfd_focus_score.
 */
mhfd_status mhfd_focus_score_backward(mhfd_plan plan, const float *d_imgs, int32_t b, int32_t h,
                                      int32_t w, const float *d_sigmas, float beta, float tau,
                                      const float *d_grad_scores, float *d_grad_imgs,
                                      float *d_grad_sigmas, int32_t *d_error, void *d_ws,
                                      size_t ws_bytes, void *stream);

/* Static text for a status code. */
const char *mhfd_status_string(mhfd_status status);

/* Description of the last failure on the calling thread ("" if none). */
const char *mhfd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MHFD_H */
