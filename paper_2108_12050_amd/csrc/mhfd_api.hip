// Host side of libmhfd: plan construction (scale grid and taps in double on
// the host), argument checks, workspace layout and the C entry points.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mhfd_internal.h"

// Scratch of mhfd_log_stack_static, for callers that cannot allocate: the
// fp32 input-range word, or the stretch histogram and levels, of one call.
// Each device holds its own copy until the process ends.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (looked up once per
// device when a plan is created there).
static __device__ __align__(256) uint32_t scratch[MHFD_STATIC_SCRATCH_BYTES / sizeof(uint32_t)];
static_assert(sizeof(int32_t) * (256 * mhfd::STRETCH_COPIES + 2) <= MHFD_STATIC_SCRATCH_BYTES,
              "the stretch histogram copies fit the static scratch");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch[kMaxDevices] = {};

// This device's address of `scratch`; `dev` must be the current device.
hipError_t static_scratch_address(int dev, uint32_t** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<uint32_t*>(ptr);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

struct mhfd_plan_s {
    int device = 0;
    int K = 0;
    std::vector<float> sigmas;   // sigma_k as float
    std::vector<int> radii;      // floor(truncate * sigma_k + 0.5)
    std::vector<int> padded;     // radius rounded up to the instantiation quantum
    std::vector<int> tap_off;    // float offset of scale k's tap block
    float truncate = 4.0f, threshold = 0.0f, overlap = 1.0f;
    int polarity = MHFD_BRIGHT, dtype = MHFD_F32;
    int max_h = 0, max_w = 0;
    int64_t max_cand = 0;
    int reach = 0;               // prune row reach, floor(sqrt(max d2max))
    int d2_top = 0;              // max d2max: bounds the prune's column search
    int n_cu = 0;                // compute units of the plan's device
    float* d_taps = nullptr;     // device tap table
    int32_t* d_d2max = nullptr;  // K x K prune table (null: pruning off)
    float* d_sigmas = nullptr;   // device copy of sigmas (float)
    size_t tap_floats = 0;
    // Split-FP16 MFMA fragment tables of the scales whose radius the
    // matrix-core kernel supports (mfma_off[k] < 0: strip kernel).
    std::vector<int> mfma_off;   // first 8-half fragment of scale k
    std::vector<float> mfma_out_scale;
    uint16_t* d_frags = nullptr;
    int stretch = 0;             // histogram stretch before the stack (u8 plans)
    int criterion = MHFD_CRITERION_LOG;  // DOG: the stack holds Gaussian planes
    // Focus-score calls: the largest sigma any scale may take (uniform cap),
    // or +inf when each scale is bounded by its own launch radius instead,
    // and every scale's launch radius (padded).
    float sigma_cap = 0.0f;
    std::vector<int> focus_padded;
    uint32_t* d_scratch = nullptr;  // this device's static scratch (mhfd_log_stack_static)
    int blur = MHFD_BLUR_DIRECT;
    // MHFD_BLUR_FFT: device tables (taps in double, radii, twiddles, the
    // spectral weights of every scale), one allocation
    void* d_fft = nullptr;
    mhfd::FftTables fft{};
};

namespace {

thread_local std::string g_last_error;

mhfd_status fail(mhfd_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mhfd_status fail(mhfd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mhfd_status hip_fail(hipError_t e, const char* what) {
    return fail(MHFD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// One-sided taps of one scale in double: g[0..R] the unit-sum sampled
// Gaussian, h[0..R] = (j^2 - V) g_j / sigma^4 with V its discrete variance.
void gauss_taps(double sigma, int R, std::vector<double>& g, std::vector<double>& h) {
    g.assign(R + 1, 0.0);
    h.assign(R + 1, 0.0);
    double z = 0.0;
    for (int j = 0; j <= R; ++j) {
        g[j] = exp(-static_cast<double>(j) * j / (2.0 * sigma * sigma));
        z += j == 0 ? g[j] : 2.0 * g[j];
    }
    double var = 0.0;
    for (int j = 0; j <= R; ++j) {
        g[j] /= z;
        var += (j == 0 ? 0.0 : 2.0) * static_cast<double>(j) * j * g[j];
    }
    const double s4 = sigma * sigma * sigma * sigma;
    for (int j = 0; j <= R; ++j) h[j] = (static_cast<double>(j) * j - var) * g[j] / s4;
}

double polarity_norm(double sigma, int polarity) {
    return (polarity == MHFD_BRIGHT ? -1.0 : 1.0) * sigma * sigma;
}

// Taps of one scale in double, then rounded to float into `dst`
// (layout documented with tap_block_floats).
void synth_taps(double sigma, int R, int P, int polarity, float* dst) {
    std::vector<double> g, h;
    gauss_taps(sigma, R, g, h);
    const double norm = polarity_norm(sigma, polarity);
    for (int j = 0; j <= P; ++j) {
        const bool in = j <= R;
        dst[j] = in ? static_cast<float>(g[j]) : 0.0f;
        dst[(P + 1) + j] = in ? static_cast<float>(h[j]) : 0.0f;
        dst[2 * (P + 1) + j] = in ? static_cast<float>(norm * g[j]) : 0.0f;
        dst[3 * (P + 1) + j] = in ? static_cast<float>(norm * h[j]) : 0.0f;
    }
}

// Fraction of the smaller disc covered by the intersection of two discs whose
// centres are d apart (lens area over pi min(ra, rb)^2).
double disc_overlap(double d, double ra, double rb) {
    if (d >= ra + rb) return 0.0;
    if (d <= fabs(ra - rb)) return 1.0;
    const double rs = ra < rb ? ra : rb;
    const double ca = (d * d + ra * ra - rb * rb) / (2.0 * d * ra);
    const double cb = (d * d + rb * rb - ra * ra) / (2.0 * d * rb);
    const double lens = ra * ra * acos(ca) + rb * rb * acos(cb) -
                        0.5 * sqrt((-d + ra + rb) * (d + ra - rb) * (d - ra + rb) * (d + ra + rb));
    return lens / (M_PI * rs * rs);
}

// Largest integer D with overlap(sqrt(D)) > theta for blob radii ra, rb, or -1.
// The overlap falls monotonically as the centres move apart, so the decision
// for integer coordinates is exactly dy^2 + dx^2 <= D.
int max_overlapping_d2(double ra, double rb, double theta) {
    if (!(disc_overlap(0.0, ra, rb) > theta)) return -1;
    long lo = 0;                                             // overlap > theta
    long hi = static_cast<long>(ceil((ra + rb) * (ra + rb))) + 1;  // overlap == 0
    while (hi - lo > 1) {
        const long mid = (lo + hi) / 2;
        if (disc_overlap(sqrt(static_cast<double>(mid)), ra, rb) > theta)
            lo = mid;
        else
            hi = mid;
    }
    return static_cast<int>(lo);
}

size_t log_stack_scratch_bytes(const mhfd_plan_s* p, int h, int w) {
    if (p->blur == MHFD_BLUR_FFT) return sizeof(float) * mhfd::fft_workspace_floats(h, w);
    if (p->stretch) return sizeof(int32_t) * (256 * mhfd::STRETCH_COPIES + 2);
    return (p->d_frags && p->dtype == MHFD_F32) ? sizeof(uint32_t) : 0;
}

struct DetectLayout {
    size_t stack, blk_n, blk_o, blk_off, pool, cand, keep, keep_off, scan_sums, ctr, maxbits,
        dog_max, dog_arg, act, total;
    int n_blk, bpr;
    int act_bx, act_by;  // activity words of the threshold-sparse stack (0: dense plans)
};

// A detection without a caller stack keeps only the above-threshold part of
// the stack (plus activity words) when every scale runs on the matrix cores,
// the criterion is the LoG's and the threshold is not negative; otherwise
// the whole stack.
bool sparse_stack(const mhfd_plan_s* p) {
    // the maxima pass reads unwritten groups as 0, which must not exceed tau
    if (p->criterion != MHFD_CRITERION_LOG || p->blur != MHFD_BLUR_DIRECT || !p->d_frags ||
        !(p->threshold >= 0.0f))
        return false;
    for (int k = 0; k < p->K; ++k)
        if (p->mfma_off[k] < 0) return false;
    return true;
}

DetectLayout detect_layout(const mhfd_plan_s* p, int h, int w) {
    DetectLayout L{};
    L.bpr = mhfd::nms_blocks_per_row(w);
    L.n_blk = h * L.bpr;
    const size_t cap = static_cast<size_t>(p->max_cand);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.stack = take(sizeof(float) * static_cast<size_t>(p->K) * h * w);
    L.blk_n = take(sizeof(int32_t) * L.n_blk);
    L.blk_o = take(sizeof(int32_t) * L.n_blk);
    L.blk_off = take(sizeof(int32_t) * (L.n_blk + 1));
    L.pool = take(sizeof(mhfd::Cand) * mhfd::nms_pool_records(L.n_blk, p->max_cand));
    L.cand = take(sizeof(mhfd::Cand) * cap);
    L.keep = take(sizeof(int32_t) * cap);
    L.keep_off = take(sizeof(int32_t) * (cap + 1));
    const int64_t longest = static_cast<int64_t>(cap) > L.n_blk ? static_cast<int64_t>(cap) : L.n_blk;
    L.scan_sums = take(sizeof(int32_t) * mhfd::scan_sums_ints(longest));
    L.ctr = take(sizeof(mhfd::DetectCounters));
    L.maxbits = take(log_stack_scratch_bytes(p, h, w));
    const bool dog = p->criterion == MHFD_CRITERION_DOG;
    L.dog_max = take(dog ? sizeof(float) * static_cast<size_t>(h) * w : 0);
    L.dog_arg = take(dog ? static_cast<size_t>(h) * w : 0);
    const bool sp = sparse_stack(p);
    L.act_bx = sp ? (w + 15) / 16 : 0;
    L.act_by = sp ? (h + 15) / 16 : 0;
    L.act = take(sizeof(uint64_t) * static_cast<size_t>(p->K) * L.act_bx * L.act_by);
    L.total = off;
    return L;
}

// FFT plan tables in one device block: the one-sided taps g_0..g_R, h_0..h_R
// of every scale (double), their offsets and radii (int), twiddles
// e^{-2 pi i k / nmax} and e^{-i pi k / (2 nmax)} (k < nmax; float2 from
// double), and the spectral weights the device computes from the taps once.
hipError_t build_fft_tables(mhfd_plan_s* p) {
    int nmax = 1;
    while (nmax < p->max_h || nmax < p->max_w) nmax <<= 1;
    std::vector<double> taps;
    std::vector<int> off(p->K), rad(p->K);
    for (int k = 0; k < p->K; ++k) {
        std::vector<double> g, h;
        gauss_taps(static_cast<double>(p->sigmas[k]), p->radii[k], g, h);
        off[k] = static_cast<int>(taps.size());
        rad[k] = p->radii[k];
        taps.insert(taps.end(), g.begin(), g.end());
        taps.insert(taps.end(), h.begin(), h.end());
        p->fft.norm[k] =
            static_cast<float>(polarity_norm(static_cast<double>(p->sigmas[k]), p->polarity));
    }
    std::vector<float2> tw(nmax), q(nmax);
    for (int k = 0; k < nmax; ++k) {
        const double a = -2.0 * M_PI * k / nmax;
        tw[k] = make_float2(static_cast<float>(cos(a)), static_cast<float>(sin(a)));
        const double b = -M_PI * k / (2.0 * nmax);
        q[k] = make_float2(static_cast<float>(cos(b)), static_cast<float>(sin(b)));
    }
    size_t o = 0;
    auto place = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t o_taps = place(sizeof(double) * taps.size());
    const size_t o_off = place(sizeof(int) * off.size());
    const size_t o_rad = place(sizeof(int) * rad.size());
    const size_t o_tw = place(sizeof(float2) * tw.size());
    const size_t o_q = place(sizeof(float2) * q.size());
    const size_t o_lam = place(sizeof(float) * 2 * static_cast<size_t>(nmax) * p->K);
    std::vector<char> blob(o_lam, 0);
    memcpy(blob.data() + o_taps, taps.data(), sizeof(double) * taps.size());
    memcpy(blob.data() + o_off, off.data(), sizeof(int) * off.size());
    memcpy(blob.data() + o_rad, rad.data(), sizeof(int) * rad.size());
    memcpy(blob.data() + o_tw, tw.data(), sizeof(float2) * tw.size());
    memcpy(blob.data() + o_q, q.data(), sizeof(float2) * q.size());
    hipError_t e = hipMalloc(&p->d_fft, o);
    if (e == hipSuccess) e = hipMemcpy(p->d_fft, blob.data(), o_lam, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    char* b = static_cast<char*>(p->d_fft);
    float* lam = reinterpret_cast<float*>(b + o_lam);
    e = mhfd::build_fft_spectra(reinterpret_cast<const double*>(b + o_taps),
                                reinterpret_cast<const int*>(b + o_off),
                                reinterpret_cast<const int*>(b + o_rad), p->K, nmax, lam, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return e;
    p->fft.lam = lam;
    p->fft.tw = reinterpret_cast<const float2*>(b + o_tw);
    p->fft.q = reinterpret_cast<const float2*>(b + o_q);
    p->fft.K = p->K;
    p->fft.nmax = nmax;
    return hipSuccess;
}

mhfd_status check_device(const mhfd_plan_s* p) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device)
        return fail(MHFD_ERR_INVALID_ARG, "plan lives on device %d but device %d is current",
                    p->device, dev);
    return MHFD_OK;
}

}  // namespace

extern "C" {

const char* mhfd_status_string(mhfd_status st) {
    switch (st) {
        case MHFD_OK: return "ok";
        case MHFD_ERR_INVALID_ARG: return "invalid argument";
        case MHFD_ERR_UNSUPPORTED: return "unsupported";
        case MHFD_ERR_WORKSPACE: return "workspace too small";
        case MHFD_ERR_HIP: return "HIP error";
        case MHFD_ERR_OOM: return "out of device memory";
    }
    return "unknown status";
}

const char* mhfd_last_error(void) { return g_last_error.c_str(); }

mhfd_status mhfd_create_plan(const mhfd_config* cfg, mhfd_plan* out) {
    g_last_error.clear();
    if (!cfg || !out) return fail(MHFD_ERR_INVALID_ARG, "null config or output pointer");
    const int K = cfg->n_scales;
    if (K < 1 || K > MHFD_MAX_SCALES)
        return fail(MHFD_ERR_INVALID_ARG, "n_scales %d outside [1, %d]", K, MHFD_MAX_SCALES);
    if (!(cfg->truncate > 0.0f) || !isfinite(cfg->truncate))
        return fail(MHFD_ERR_INVALID_ARG, "truncate must be positive and finite");
    if (!isfinite(cfg->threshold)) return fail(MHFD_ERR_INVALID_ARG, "threshold must be finite");
    if (!(cfg->overlap >= 0.0f) || !isfinite(cfg->overlap))
        return fail(MHFD_ERR_INVALID_ARG, "overlap must be >= 0 and finite");
    if (cfg->polarity != MHFD_BRIGHT && cfg->polarity != MHFD_DARK)
        return fail(MHFD_ERR_INVALID_ARG, "unknown polarity %d", cfg->polarity);
    if (cfg->in_dtype != MHFD_F32 && cfg->in_dtype != MHFD_U8)
        return fail(MHFD_ERR_INVALID_ARG, "unknown input dtype %d", cfg->in_dtype);
    if (cfg->max_h < 1 || cfg->max_w < 1)
        return fail(MHFD_ERR_INVALID_ARG, "max_h and max_w must be >= 1");
    if (static_cast<int64_t>(cfg->max_h) * cfg->max_w > (int64_t(1) << 31) / 4)
        return fail(MHFD_ERR_UNSUPPORTED, "max_h * max_w above 2^29 pixels");
    if (cfg->max_candidates < 0) return fail(MHFD_ERR_INVALID_ARG, "max_candidates < 0");
    if (cfg->criterion != MHFD_CRITERION_LOG && cfg->criterion != MHFD_CRITERION_DOG)
        return fail(MHFD_ERR_INVALID_ARG, "unknown criterion %d", cfg->criterion);
    if (cfg->criterion == MHFD_CRITERION_DOG && K < 2)
        return fail(MHFD_ERR_INVALID_ARG, "the DoG criterion needs at least two scales");
    if (cfg->criterion == MHFD_CRITERION_DOG && cfg->overlap < 1.0f)
        return fail(MHFD_ERR_UNSUPPORTED, "the DoG criterion has no overlap pruning (overlap >= 1)");
    if (cfg->stretch != 0 && cfg->stretch != 1)
        return fail(MHFD_ERR_INVALID_ARG, "stretch must be 0 or 1");
    if (cfg->stretch && cfg->in_dtype != MHFD_U8)
        return fail(MHFD_ERR_UNSUPPORTED, "the histogram stretch is built for 8-bit plans");
    if (!(cfg->sigma_cap >= 0.0f) || !isfinite(cfg->sigma_cap))
        return fail(MHFD_ERR_INVALID_ARG, "sigma_cap must be >= 0 and finite");
    if (cfg->blur != MHFD_BLUR_DIRECT && cfg->blur != MHFD_BLUR_FFT)
        return fail(MHFD_ERR_INVALID_ARG, "unknown blur %d", cfg->blur);
    const bool fft = cfg->blur == MHFD_BLUR_FFT;
    if (fft && (cfg->criterion != MHFD_CRITERION_LOG || cfg->stretch))
        return fail(MHFD_ERR_UNSUPPORTED, "the FFT blur takes LoG plans without the stretch");
    if (fft && (cfg->max_h > MHFD_MAX_FFT_SIZE || cfg->max_w > MHFD_MAX_FFT_SIZE))
        return fail(MHFD_ERR_UNSUPPORTED, "the FFT blur takes tiles up to %d x %d",
                    MHFD_MAX_FFT_SIZE, MHFD_MAX_FFT_SIZE);

    std::vector<float> sig(K);
    if (cfg->sigmas) {
        for (int k = 0; k < K; ++k) sig[k] = cfg->sigmas[k];
    } else if (K == 1) {
        sig[0] = cfg->sigma_min;
    } else {
        // section 2.2: t_i = min_t + (i - 1) delta_t, delta_t = (max_t - min_t) / n, K = n + 1
        const double a = cfg->sigma_min, b = cfg->sigma_max;
        const double dt = (b - a) / (K - 1);
        for (int k = 0; k < K; ++k) sig[k] = static_cast<float>(a + k * dt);
    }
    for (int k = 0; k < K; ++k) {
        if (!(sig[k] > 0.0f) || !isfinite(sig[k]))
            return fail(MHFD_ERR_INVALID_ARG, "sigma[%d] = %g is not positive and finite", k,
                        static_cast<double>(sig[k]));
        if (k > 0 && !(sig[k] > sig[k - 1]))
            return fail(MHFD_ERR_INVALID_ARG, "sigmas must be strictly increasing (sigma[%d])", k);
    }

    mhfd_plan_s* p = new (std::nothrow) mhfd_plan_s();
    if (!p) return fail(MHFD_ERR_OOM, "host allocation of the plan failed");
    p->K = K;
    p->sigmas = sig;
    p->truncate = cfg->truncate;
    p->threshold = cfg->threshold;
    p->overlap = cfg->overlap;
    p->polarity = cfg->polarity;
    p->dtype = cfg->in_dtype;
    p->max_h = cfg->max_h;
    p->max_w = cfg->max_w;
    p->stretch = cfg->stretch;
    p->criterion = cfg->criterion;
    p->blur = cfg->blur;
    int64_t dc = static_cast<int64_t>(cfg->max_h) * cfg->max_w / 64;
    p->max_cand = cfg->max_candidates > 0 ? cfg->max_candidates : (dc > 65536 ? dc : 65536);
    if (p->max_cand > (int64_t(1) << 30)) {
        delete p;
        return fail(MHFD_ERR_UNSUPPORTED, "max_candidates above 2^30");
    }
    size_t off = 0;
    for (int k = 0; k < K; ++k) {
        const int R = static_cast<int>(floor(static_cast<double>(p->truncate) * sig[k] + 0.5));
        const int rmax = fft ? MHFD_MAX_FFT_RADIUS : MHFD_MAX_RADIUS;
        if (R > rmax) {
            delete p;
            return fail(MHFD_ERR_UNSUPPORTED, "radius %d of sigma %g exceeds %d", R,
                        static_cast<double>(sig[k]), rmax);
        }
        if ((cfg->stretch || cfg->criterion == MHFD_CRITERION_DOG) && !mhfd::mfma_radius_ok(R)) {
            delete p;
            return fail(MHFD_ERR_UNSUPPORTED,
                        "the histogram stretch and the DoG criterion need every radius on the "
                        "matrix-core path (radius %d of sigma %g)", R, static_cast<double>(sig[k]));
        }
        const int P = mhfd::padded_radius(R < 1 ? 1 : R);
        p->radii.push_back(R);
        p->padded.push_back(P);
        p->tap_off.push_back(static_cast<int>(off));
        off += mhfd::tap_block_floats(P);
    }
    p->tap_floats = off;
    if (cfg->sigma_cap > 0.0f) {
        // uniform cap: every scale's halo sized for the cap's radius
        const float cap = cfg->sigma_cap;
        const double rc = floor(static_cast<double>(p->truncate) * cap + 0.5);
        if (cap < sig[K - 1] || rc > MHFD_MAX_RADIUS) {
            delete p;
            return fail(cap < sig[K - 1] ? MHFD_ERR_INVALID_ARG : MHFD_ERR_UNSUPPORTED,
                        "sigma_cap %g must be >= the largest sigma %g and give a radius <= %d",
                        static_cast<double>(cap), static_cast<double>(sig[K - 1]),
                        MHFD_MAX_RADIUS);
        }
        p->sigma_cap = cap;
        const int rcap = static_cast<int>(rc);
        p->focus_padded.assign(K, mhfd::padded_radius(rcap < 1 ? 1 : rcap));
    } else {
        // each scale within its own padded plan radius
        p->sigma_cap = INFINITY;
        p->focus_padded = p->padded;
    }
    // Blob radius sqrt(2) sigma; prune table in double.
    std::vector<int32_t> d2(static_cast<size_t>(K) * K, -1);
    int d2_top = 0;
    const bool prune = p->overlap < 1.0f;
    if (prune) {
        const double sq2 = sqrt(2.0);
        for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b) {
                d2[a * K + b] = max_overlapping_d2(sq2 * sig[a], sq2 * sig[b],
                                                   static_cast<double>(p->overlap));
                if (d2[a * K + b] > d2_top) d2_top = d2[a * K + b];
            }
    }
    p->d2_top = d2_top;
    p->reach = static_cast<int>(floor(sqrt(static_cast<double>(d2_top))));
    std::vector<float> host(off, 0.0f);
    for (int k = 0; k < K; ++k)
        synth_taps(static_cast<double>(sig[k]), p->radii[k], p->padded[k], p->polarity,
                   host.data() + p->tap_off[k]);
    // Matrix-core fragment tables: u8 codes 0..255 (intensity code / 255), or
    // fp32 values scaled on the device so that max |I| < 2^14.
    std::vector<uint16_t> frags;
    p->mfma_off.assign(K, -1);
    p->mfma_out_scale.assign(K, 0.0f);
    const bool u8 = p->dtype == MHFD_U8;
    {
        for (int k = 0; k < K; ++k) {
            const int R = p->radii[k];
            if (!mhfd::mfma_radius_ok(R) || p->blur == MHFD_BLUR_FFT) continue;
            std::vector<double> g, h;
            gauss_taps(static_cast<double>(sig[k]), R, g, h);
            const size_t at = frags.size();
            frags.resize(at + mhfd::mfma_frag_halves(R));
            p->mfma_off[k] = static_cast<int>(at / 8);
            // DoG criterion: Gaussian planes.  With g in place of h both
            // separable terms are g(x) g(y), so norm 1/2 gives L exactly.
            const bool dog = p->criterion == MHFD_CRITERION_DOG;
            p->mfma_out_scale[k] = mhfd::mfma_build_frags(
                g.data(), dog ? g.data() : h.data(), R,
                dog ? 0.5 : polarity_norm(static_cast<double>(sig[k]), p->polarity),
                u8 ? 255.0 : 1.0, u8 ? 255.0 : 16384.0, frags.data() + at);
        }
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = static_scratch_address(p->device, &p->d_scratch);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "device query");
    }
    e = hipMalloc(reinterpret_cast<void**>(&p->d_taps), sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_sigmas), sizeof(float) * K);
    if (e == hipSuccess && prune)
        e = hipMalloc(reinterpret_cast<void**>(&p->d_d2max), sizeof(int32_t) * K * K);
    if (e == hipSuccess && !frags.empty())
        e = hipMalloc(reinterpret_cast<void**>(&p->d_frags), sizeof(uint16_t) * frags.size());
    if (e != hipSuccess) {
        hipFree(p->d_taps);
        hipFree(p->d_sigmas);
        hipFree(p->d_d2max);
        hipFree(p->d_frags);
        delete p;
        return fail(MHFD_ERR_OOM, "plan tables: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_taps, host.data(), sizeof(float) * off, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_sigmas, sig.data(), sizeof(float) * K, hipMemcpyHostToDevice);
    if (e == hipSuccess && prune)
        e = hipMemcpy(p->d_d2max, d2.data(), sizeof(int32_t) * K * K, hipMemcpyHostToDevice);
    if (e == hipSuccess && !frags.empty())
        e = hipMemcpy(p->d_frags, frags.data(), sizeof(uint16_t) * frags.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(p->d_taps);
        hipFree(p->d_sigmas);
        hipFree(p->d_d2max);
        hipFree(p->d_frags);
        delete p;
        return hip_fail(e, "copy of the plan tables");
    }
    if (p->blur == MHFD_BLUR_FFT && (e = build_fft_tables(p)) != hipSuccess) {
        mhfd_destroy_plan(p);
        return hip_fail(e, "FFT plan tables");
    }
    *out = p;
    return MHFD_OK;
}

mhfd_status mhfd_destroy_plan(mhfd_plan p) {
    if (!p) return MHFD_OK;
    hipFree(p->d_taps);
    hipFree(p->d_sigmas);
    hipFree(p->d_d2max);
    hipFree(p->d_frags);
    hipFree(p->d_fft);
    delete p;
    return MHFD_OK;
}

int32_t mhfd_plan_scales(mhfd_plan p, float* sigmas, int32_t* radii) {
    if (!p) return -1;
    for (int k = 0; k < p->K; ++k) {
        if (sigmas) sigmas[k] = p->sigmas[k];
        if (radii) radii[k] = p->radii[k];
    }
    return p->K;
}

size_t mhfd_detect_workspace_size(mhfd_plan p, int32_t h, int32_t w) {
    if (!p || h < 1 || w < 1 || h > p->max_h || w > p->max_w) return 0;
    return detect_layout(p, h, w).total;
}

}  // extern "C"

namespace {

mhfd_status check_image(const mhfd_plan_s* p, const void* d_img, int32_t h, int32_t w,
                        int64_t pitch) {
    if (!p) return fail(MHFD_ERR_INVALID_ARG, "null plan");
    if (!d_img) return fail(MHFD_ERR_INVALID_ARG, "null image");
    if (h < 1 || w < 1) return fail(MHFD_ERR_INVALID_ARG, "image %d x %d is empty", h, w);
    if (h > p->max_h || w > p->max_w)
        return fail(MHFD_ERR_INVALID_ARG, "image %d x %d exceeds the plan's %d x %d", h, w,
                    p->max_h, p->max_w);
    if (pitch < w) return fail(MHFD_ERR_INVALID_ARG, "pitch %lld < width %d", (long long)pitch, w);
    if (p->dtype == MHFD_F32 && reinterpret_cast<uintptr_t>(d_img) % 4)
        return fail(MHFD_ERR_INVALID_ARG, "float image not 4-byte aligned");
    if (p->blur == MHFD_BLUR_FFT && (!mhfd::fft_size_ok(h) || !mhfd::fft_size_ok(w)))
        return fail(MHFD_ERR_UNSUPPORTED, "the FFT blur takes power-of-two sides (image %d x %d)",
                    h, w);
    return MHFD_OK;
}

mhfd_status check_outputs(const mhfd_plan_s* p, int32_t h, int32_t w, const mhfd_blob* d_blobs,
                          int32_t capacity, const mhfd_result* d_result, const void* d_ws,
                          size_t ws_bytes, DetectLayout* L) {
    if (!d_result || !d_ws) return fail(MHFD_ERR_INVALID_ARG, "null result or workspace");
    if (capacity < 0) return fail(MHFD_ERR_INVALID_ARG, "capacity < 0");
    if (capacity > 0 && !d_blobs) return fail(MHFD_ERR_INVALID_ARG, "null blob buffer");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(MHFD_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    *L = detect_layout(p, h, w);
    if (ws_bytes < L->total)
        return fail(MHFD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L->total);
    return MHFD_OK;
}

// Per radius class, the launch covering `scales` (largest radius first):
// tap_off(k) gives the tap block of scale k, plane(k) its output plane.
// Segment heights: every segment recomputes a 2R-row halo of row-pass
// results, so a scale gets about 16R rows per workgroup (halo overhead near
// 10%), halved while the launch would have fewer than ~3 workgroups per
// resident slot.
template <typename TapOff, typename Plane, typename Pad>
std::vector<std::pair<int, mhfd::StackLaunch>> make_launches(const mhfd_plan_s* p, int h, int w,
                                                             const std::vector<int>& scales,
                                                             TapOff tap_off, Plane plane, Pad pad) {
    const int tw = mhfd::log_strip_width();
    const int ch = mhfd::log_chunk_rows();
    const int strips = (w + tw - 1) / tw;
    const int target = 6 * (p->n_cu > 0 ? p->n_cu : 256);
    std::vector<std::pair<int, mhfd::StackLaunch>> out;
    for (int cls = 2; cls >= 0; --cls) {
        std::vector<int> ks;
        for (int k : scales)
            if (mhfd::log_radius_class(pad(k)) == cls) ks.push_back(k);
        if (ks.empty()) continue;
        std::sort(ks.begin(), ks.end(), [&](int a, int b) {
            return pad(a) != pad(b) ? pad(a) > pad(b) : a < b;
        });
        const int hr = (h + ch - 1) / ch * ch;
        std::vector<int> seg(ks.size());
        for (size_t i = 0; i < ks.size(); ++i) {
            int sgr = 16 * pad(ks[i]);
            sgr = sgr < 2 * ch ? 2 * ch : (sgr > 1024 ? 1024 : sgr);
            sgr = (sgr + ch - 1) / ch * ch;
            seg[i] = sgr < hr ? sgr : hr;
        }
        auto blocks = [&]() {
            long long n = 0;
            for (size_t i = 0; i < ks.size(); ++i) n += static_cast<long long>(strips) * ((h + seg[i] - 1) / seg[i]);
            return n;
        };
        while (blocks() < target) {
            bool shrunk = false;
            for (auto& sgr : seg)
                if (sgr > ch) {
                    sgr = ((sgr / 2 + ch - 1) / ch) * ch;
                    shrunk = true;
                }
            if (!shrunk) break;
        }
        mhfd::StackLaunch L{};
        L.strips = strips;
        int begin = 0;
        for (size_t i = 0; i < ks.size(); ++i) {
            const int k = ks[i];
            mhfd::StackScale& sc = L.sc[L.n++];
            sc.radius = pad(k);
            sc.tap_off = tap_off(k);
            sc.plane = plane(k);
            sc.seg_rows = seg[i];
            sc.block_begin = begin;
            sc.n_blocks = strips * ((h + seg[i] - 1) / seg[i]);
            begin += sc.n_blocks;
        }
        out.emplace_back(cls, L);
    }
    return out;
}

int launch_blocks(const mhfd::StackLaunch& L) {
    int n = 0;
    for (int i = 0; i < L.n; ++i) n += L.sc[i].n_blocks;
    return n;
}

std::vector<int> all_scales(const mhfd_plan_s* p) {
    std::vector<int> v(p->K);
    for (int k = 0; k < p->K; ++k) v[k] = k;
    return v;
}

// (nkr, nkc) shapes of the plan's matrix-core scales, costliest first.
std::vector<std::pair<int, int>> mfma_shapes(const mhfd_plan_s* p) {
    std::vector<std::pair<int, int>> shapes;
    if (!p->d_frags) return shapes;
    for (int k = 0; k < p->K; ++k) {
        if (p->mfma_off[k] < 0) continue;
        const mhfd::MfmaShape m = mhfd::mfma_shape(p->radii[k]);
        const std::pair<int, int> key(m.nkr, m.nkc);
        if (std::find(shapes.begin(), shapes.end(), key) == shapes.end()) shapes.push_back(key);
    }
    std::sort(shapes.begin(), shapes.end(), [](const std::pair<int, int>& a,
                                               const std::pair<int, int>& b) {
        return a.second != b.second ? a.second > b.second : a.first > b.first;
    });
    return shapes;
}

// Work counter of a shape in the batched launch: the shapes are (n, n),
// n = 1..4.
int mfma_slot(const std::pair<int, int>& key) {
    if (key.first != key.second || key.first < 1 || key.first > 4) return -1;
    return key.first - 1;
}

// Matrix-core launches of the scales that have fragment tables, one per
// (nkr, nkc) instantiation, largest first.  A wave computes one 16-column
// tile over a segment of rows and first recomputes the intermediate blocks
// its ring holds; segments are 1024 rows, halved while a launch has fewer
// than 8 waves per compute unit.
std::vector<std::pair<std::pair<int, int>, mhfd::MfmaLaunch>> mfma_launches(const mhfd_plan_s* p,
                                                                             int h, int w) {
    std::vector<std::pair<std::pair<int, int>, mhfd::MfmaLaunch>> out;
    if (!p->d_frags) return out;
    const int tiles_x = mhfd::mfma_wave_tiles(w);
    const int mw = mhfd::mfma_waves_per_block();
    const int groups_x = (tiles_x + mw - 1) / mw;
    // at least 8 waves per CU, as few row segments as that allows: every
    // segment repeats the ring's warm-up and the wave's set-up
    const long long target = 8LL * (p->n_cu > 0 ? p->n_cu : 256);
    const int hr = (h + 15) / 16 * 16;
    for (const auto& key : mfma_shapes(p)) {
        std::vector<int> ks;
        for (int k = 0; k < p->K; ++k) {
            if (p->mfma_off[k] < 0) continue;
            const mhfd::MfmaShape m = mhfd::mfma_shape(p->radii[k]);
            if (m.nkr == key.first && m.nkc == key.second) ks.push_back(k);
        }
        int seg = 1024 < hr ? 1024 : hr;
        auto waves = [&]() {
            return static_cast<long long>(ks.size()) * tiles_x * ((h + seg - 1) / seg);
        };
        while (waves() < target && seg > 16) seg = (seg / 2 + 15) / 16 * 16;
        mhfd::MfmaLaunch L{};
        L.tiles_x = tiles_x;
        L.groups_x = groups_x;
        int begin = 0;
        for (int k : ks) {
            const mhfd::MfmaShape m = mhfd::mfma_shape(p->radii[k]);
            mhfd::MfmaScale& sc = L.sc[L.n++];
            sc.rw8 = m.rw8;
            sc.rwc = m.rwc;
            sc.frag_off = p->mfma_off[k];
            sc.plane = k;
            sc.seg_rows = seg;
            sc.block_begin = begin;
            sc.n_blocks = groups_x * ((h + seg - 1) / seg);
            sc.out_scale = p->mfma_out_scale[k];
            begin += sc.n_blocks;
        }
        out.emplace_back(key, L);
    }
    return out;
}

// Bytes of scratch the stack needs: the max |I| word of fp32 plans with
// matrix-core scales; the global copies of the 256-bin histogram and the two
// levels of stretch plans.
size_t log_stack_scratch(const mhfd_plan_s* p, int h, int w) {
    return log_stack_scratch_bytes(p, h, w);
}

mhfd_status enqueue_log_stack(const mhfd_plan_s* p, const void* d_img, int h, int w,
                              int64_t pitch, float* stack, uint32_t* maxbits, hipStream_t s,
                              const mhfd::ActOut& act = mhfd::ActOut{nullptr, 0, 0, 0.0f}) {
    if (p->blur == MHFD_BLUR_FFT) {
        hipError_t e = mhfd::launch_fft_log_stack(p->fft, p->dtype, d_img, h, w, pitch, stack,
                                                  reinterpret_cast<float*>(maxbits), s);
        if (e != hipSuccess) return hip_fail(e, "LoG stack (FFT) launch");
        return MHFD_OK;
    }
    std::vector<int> strip_scales;
    for (int k = 0; k < p->K; ++k)
        if (p->mfma_off.empty() || p->mfma_off[k] < 0) strip_scales.push_back(k);
    const auto mls = mfma_launches(p, h, w);
    // fp32: max |I| word; stretch: histogram copies (8 x 256 counts), then {low, high}
    const uint32_t* range = nullptr;
    if (!mls.empty() && p->dtype == MHFD_F32) {
        hipError_t e = mhfd::launch_absmax(static_cast<const float*>(d_img), h, w, pitch, maxbits, s);
        if (e != hipSuccess) return hip_fail(e, "input range pass");
        range = maxbits;
    }
    if (p->stretch) {
        int32_t* copies = reinterpret_cast<int32_t*>(maxbits);
        int32_t* levels = copies + 256 * mhfd::STRETCH_COPIES;
        hipError_t e = mhfd::launch_stretch_levels(static_cast<const uint8_t*>(d_img), h, w, pitch,
                                                   copies, mhfd::STRETCH_COPIES, nullptr, levels,
                                                   p->n_cu, s);
        if (e != hipSuccess) return hip_fail(e, "histogram stretch levels");
        range = reinterpret_cast<const uint32_t*>(levels);
    }
    for (const auto& ml : mls) {
        hipError_t e = mhfd::launch_log_mfma(p->dtype, p->stretch, ml.first.first, ml.first.second,
                                             d_img, h, w, pitch, range, p->d_frags, ml.second,
                                             stack, static_cast<long long>(h) * w, act, s);
        if (e != hipSuccess) return hip_fail(e, "LoG stack (matrix cores) launch");
    }
    auto launches = make_launches(
        p, h, w, strip_scales, [&](int k) { return p->tap_off[k]; }, [](int k) { return k; },
        [&](int k) { return p->padded[k]; });
    mhfd::StackIO io{};
    io.out = stack;
    io.plane_stride = static_cast<long long>(h) * w;
    for (auto& cl : launches) {
        hipError_t e = mhfd::launch_log_class(cl.first, p->dtype, mhfd::EPI_STORE, d_img, h, w,
                                              pitch, 1, p->d_taps, cl.second, io, s);
        if (e != hipSuccess) return hip_fail(e, "LoG stack launch");
    }
    return MHFD_OK;
}

mhfd_status enqueue_tail(const mhfd_plan_s* p, const float* stack, int h, int w,
                         const DetectLayout& L, char* base, mhfd_blob* d_blobs, int capacity,
                         mhfd_result* d_result, hipStream_t s, const uint64_t* act = nullptr) {
    mhfd::DetectWorkspace ws;
    if (act) {
        ws.act = act;
        ws.act_bx = (w + 15) / 16;
        ws.act_by = (h + 15) / 16;
    }
    ws.stack = stack;
    ws.blk_n = reinterpret_cast<int32_t*>(base + L.blk_n);
    ws.blk_o = reinterpret_cast<int32_t*>(base + L.blk_o);
    ws.blk_off = reinterpret_cast<int32_t*>(base + L.blk_off);
    ws.pool = reinterpret_cast<mhfd::Cand*>(base + L.pool);
    ws.cand = reinterpret_cast<mhfd::Cand*>(base + L.cand);
    ws.keep = reinterpret_cast<int32_t*>(base + L.keep);
    ws.keep_off = reinterpret_cast<int32_t*>(base + L.keep_off);
    ws.scan_sums = reinterpret_cast<int32_t*>(base + L.scan_sums);
    ws.ctr = reinterpret_cast<mhfd::DetectCounters*>(base + L.ctr);
    ws.cap = p->max_cand;
    ws.n_blk = L.n_blk;
    ws.blk_per_row = L.bpr;
    if (p->criterion == MHFD_CRITERION_DOG) {
        // largest DoG over scale and its argmax, then the tail on that plane
        float* M = reinterpret_cast<float*>(base + L.dog_max);
        uint8_t* arg = reinterpret_cast<uint8_t*>(base + L.dog_arg);
        hipError_t e = mhfd::launch_dog(stack, p->K, p->d_sigmas, h, w, M, arg, s);
        if (e != hipSuccess) return hip_fail(e, "DoG launch");
        ws.stack = M;
        e = mhfd::launch_detect_tail(ws, 1, h, w, p->threshold, nullptr, 0, 0, p->d_sigmas,
                                     d_blobs, capacity, d_result, s);
        if (e == hipSuccess) e = mhfd::launch_dog_label(d_blobs, capacity, d_result, arg, w,
                                                        p->d_sigmas, s);
        if (e != hipSuccess) return hip_fail(e, "detection launch");
        return MHFD_OK;
    }
    hipError_t e = mhfd::launch_detect_tail(ws, p->K, h, w, p->threshold, p->d_d2max, p->reach,
                                            p->d2_top, p->d_sigmas, d_blobs, capacity,
                                            d_result, s);
    if (e != hipSuccess) return hip_fail(e, "detection launch");
    return MHFD_OK;
}

struct FocusLayout {
    size_t taps, partial, rplane, dplane, cot, frags, scales, maxbits, total;
    int cot_stride;  // sigma-gradient partials per scale
    mhfd::SoftTapLayout lay;
    int fwd_blocks;  // workgroups per image over every class launch (strip form)
    bool mfma;       // matrix-core form
    mhfd::SoftFragLayout fl;
};

// The soft score runs on the matrix cores when every scale's launch radius
// is within their limit (else on the strip kernel).
bool soft_mfma_ok(const mhfd_plan_s* p) {
    for (int k = 0; k < p->K; ++k) {
        const int P = p->focus_padded[k];
        if (!mhfd::mfma_radius_ok(P)) return false;
        const mhfd::MfmaShape m = mhfd::mfma_shape(P);
        if (m.nkr != m.nkc || m.nkr < 1 || m.nkr > mhfd::MFMA_SHAPES) return false;
    }
    return true;
}

// Matrix-core launches of tap set `set` over scales ks for a batch of b
// images, one per shape: (nkr, launch).
std::vector<std::pair<int, mhfd::MfmaLaunch>> soft_mfma_launches(const mhfd_plan_s* p,
                                                                 const mhfd::SoftFragLayout& fl,
                                                                 int b, int h, int w,
                                                                 const std::vector<int>& ks,
                                                                 int set, int set2 = -1) {
    std::vector<std::pair<int, mhfd::MfmaLaunch>> out;
    const int tiles_x = mhfd::mfma_wave_tiles(w);
    const int mw = mhfd::mfma_waves_per_block();
    const int groups_x = (tiles_x + mw - 1) / mw;
    const long long target = 8LL * (p->n_cu > 0 ? p->n_cu : 256);
    const int hr = (h + 15) / 16 * 16;
    for (int a = 1; a <= mhfd::MFMA_SHAPES; ++a) {
        std::vector<int> sel;
        for (int k : ks)
            if (fl.nkr[k] == a) sel.push_back(k);
        if (sel.empty()) continue;
        int seg = 1024 < hr ? 1024 : hr;
        auto waves = [&]() {
            return static_cast<long long>(sel.size()) * b * tiles_x * ((h + seg - 1) / seg);
        };
        while (waves() < target && seg > 16) seg = (seg / 2 + 15) / 16 * 16;
        mhfd::MfmaLaunch L{};
        L.tiles_x = tiles_x;
        L.groups_x = groups_x;
        L.img_stride = static_cast<long long>(h) * w;
        L.out_stride = static_cast<long long>(h) * w;
        int begin = 0;
        for (int k : sel) {
            mhfd::MfmaScale& sc = L.sc[L.n++];
            sc.rw8 = fl.rw8[k];
            sc.rwc = fl.rwc[k];
            sc.frag_off = static_cast<int>((fl.off[k] + static_cast<long long>(set) * fl.halves[k]) / 8);
            sc.plane = 0;
            sc.seg_rows = seg;
            sc.block_begin = begin;
            sc.n_blocks = groups_x * ((h + seg - 1) / seg);
            sc.out_scale = 0.0f;
            sc.dev_scale_idx = 4 * k + set;
            if (set2 >= 0) {  // EPI_DUAL: the second set's columns on the same row pass
                sc.frag_off2 =
                    static_cast<int>((fl.off[k] + static_cast<long long>(set2) * fl.halves[k]) / 8);
                sc.dev_scale_idx2 = 4 * k + set2;
            }
            begin += sc.n_blocks;
        }
        out.emplace_back(a, L);
    }
    return out;
}

int mfma_launch_blocks(const mhfd::MfmaLaunch& L) {
    int n = 0;
    for (int i = 0; i < L.n; ++i) n += L.sc[i].n_blocks;
    return n;
}

FocusLayout focus_layout(const mhfd_plan_s* p, int b, int h, int w) {
    FocusLayout F{};
    F.lay.K = p->K;
    F.lay.truncate = p->truncate;
    F.lay.sigma_cap = p->sigma_cap;
    int off = 0;
    for (int k = 0; k < p->K; ++k) {
        F.lay.padded[k] = p->focus_padded[k];
        F.lay.offset[k] = off;
        off += mhfd::SOFT_SETS * 4 * (p->focus_padded[k] + 1);
    }
    auto launches = make_launches(
        p, h, w, all_scales(p), [](int) { return 0; }, [](int k) { return k; },
        [&](int k) { return p->focus_padded[k]; });
    F.fwd_blocks = 0;
    for (auto& cl : launches) F.fwd_blocks += launch_blocks(cl.second);
    size_t partials = static_cast<size_t>(F.fwd_blocks) * b;
    long long frag_halves = 0;
    F.mfma = soft_mfma_ok(p);
    if (F.mfma) {
        F.fl.K = p->K;
        for (int k = 0; k < p->K; ++k) {
            const mhfd::MfmaShape m = mhfd::mfma_shape(p->focus_padded[k]);
            F.fl.nkr[k] = m.nkr;
            F.fl.nkc[k] = m.nkc;
            F.fl.rw8[k] = m.rw8;
            F.fl.rwc[k] = m.rwc;
            F.fl.halves[k] = static_cast<int>(mhfd::mfma_frag_halves(p->focus_padded[k]));
            F.fl.off[k] = frag_halves;
            frag_halves += static_cast<long long>(mhfd::SOFT_SETS) * F.fl.halves[k];
        }
        size_t waves = 0;
        for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, all_scales(p), mhfd::SOFT_FWD))
            waves += static_cast<size_t>(mfma_launch_blocks(ml.second)) *
                     mhfd::mfma_waves_per_block() * b;
        if (waves > partials) partials = waves;
    }
    F.cot_stride = mhfd::soft_cotangent_blocks(b);
    if (F.mfma) {  // the cotangent epilogue: one partial per wave of each scale's launch
        F.cot_stride = 0;
        for (int k = 0; k < p->K; ++k)
            for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, {k}, mhfd::SOFT_D2))
                F.cot_stride = std::max(F.cot_stride, mfma_launch_blocks(ml.second) *
                                                          mhfd::mfma_waves_per_block() * b);
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    F.taps = take(sizeof(float) * off);
    F.partial = take(sizeof(double) * partials);
    F.rplane = take(sizeof(float) * static_cast<size_t>(b) * h * w);
    F.dplane = take(sizeof(float) * static_cast<size_t>(b) * h * w);
    F.cot = take(sizeof(double) * static_cast<size_t>(p->K) * F.cot_stride);
    F.frags = take(sizeof(uint16_t) * static_cast<size_t>(frag_halves));
    F.scales = take(sizeof(float) * 4 * p->K);
    F.maxbits = take(sizeof(uint32_t) * 2 * static_cast<size_t>(b));
    F.total = o;
    return F;
}

mhfd_status check_focus(const mhfd_plan_s* p, const float* d_imgs, int b, int h, int w,
                        const float* d_sigmas, float beta, float tau, const void* d_ws,
                        size_t ws_bytes) {
    if (!p) return fail(MHFD_ERR_INVALID_ARG, "null plan");
    if (p->stretch || p->criterion != MHFD_CRITERION_LOG || p->blur != MHFD_BLUR_DIRECT)
        return fail(MHFD_ERR_UNSUPPORTED, "the focus score takes plain LoG plans only");
    if (!d_imgs || !d_sigmas || !d_ws) return fail(MHFD_ERR_INVALID_ARG, "null pointer argument");
    if (b < 1 || h < 1 || w < 1) return fail(MHFD_ERR_INVALID_ARG, "empty batch %d x %d x %d", b, h, w);
    if (h > p->max_h || w > p->max_w)
        return fail(MHFD_ERR_INVALID_ARG, "image %d x %d exceeds the plan's %d x %d", h, w,
                    p->max_h, p->max_w);
    if (!(beta > 0.0f) || !isfinite(beta) || !isfinite(tau))
        return fail(MHFD_ERR_INVALID_ARG, "beta must be positive and finite, tau finite");
    if (reinterpret_cast<uintptr_t>(d_imgs) % 4 || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(MHFD_ERR_INVALID_ARG, "misaligned image or workspace");
    const size_t need = focus_layout(p, b, h, w).total;
    if (ws_bytes < need)
        return fail(MHFD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    return MHFD_OK;
}

struct BatchLayout {
    size_t stack, tiles, ctr, blk_n, blk_o, blk_off, pool, cand, keep, keep_off, scan_sums, maxbits,
        act, total;
    int n_blk_bound;
    int64_t cap;
};

bool batch_layout(const mhfd_plan_s* p, int n, int64_t max_pixels, BatchLayout* L) {
    if (n < 1 || n > MHFD_MAX_BATCH || max_pixels < 1 || max_pixels > (int64_t(1) << 31) - 1)
        return false;
    // maxima cells: h * ceil(w / 64) <= h w / 64 + h per tile
    const int64_t nbb = max_pixels / 64 + static_cast<int64_t>(n) * (p->max_h + 1);
    if (nbb > (int64_t(1) << 30)) return false;
    L->n_blk_bound = static_cast<int>(nbb);
    int64_t cap = p->max_cand * n;
    if (cap > (int64_t(1) << 30)) cap = int64_t(1) << 30;
    L->cap = cap;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    // every tile's planes start on a float4: up to 3 floats of padding each
    L->stack = take(sizeof(float) * (static_cast<size_t>(p->K) * max_pixels + 4 * static_cast<size_t>(n)));
    L->tiles = take(sizeof(mhfd::BatchTile) * n);
    L->ctr = take(sizeof(mhfd::BatchCounters));
    L->blk_n = take(sizeof(int32_t) * nbb);
    L->blk_o = take(sizeof(int32_t) * nbb);
    L->blk_off = take(sizeof(int32_t) * (nbb + 1));
    L->pool = take(sizeof(mhfd::Cand) * mhfd::nms_pool_records(static_cast<int>(nbb), cap));
    L->cand = take(sizeof(mhfd::Cand) * cap);
    L->keep = take(sizeof(int32_t) * cap);
    L->keep_off = take(sizeof(int32_t) * (cap + 1));
    L->scan_sums = take(sizeof(int32_t) * mhfd::scan_sums_ints(nbb > cap ? nbb : cap));
    L->maxbits = take(sizeof(uint32_t) * n);
    L->act = take(sparse_stack(p) ? sizeof(uint64_t) * mhfd::batch_act_words(
                                        p->K, n, max_pixels, p->max_h, p->max_w) : 0);
    L->total = off;
    return true;
}

}  // namespace

extern "C" {

size_t mhfd_log_stack_workspace_size(mhfd_plan p, int32_t h, int32_t w) {
    if (!p || h < 1 || w < 1 || h > p->max_h || w > p->max_w) return 0;
    return log_stack_scratch(p, h, w);
}

mhfd_status mhfd_log_stack(mhfd_plan p, const void* d_img, int32_t h, int32_t w, int64_t pitch,
                           float* d_stack, void* d_ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_img, h, w, pitch);
    if (st != MHFD_OK) return st;
    if (!d_stack) return fail(MHFD_ERR_INVALID_ARG, "null stack");
    const size_t need = log_stack_scratch(p, h, w);
    if (need) {
        if (!d_ws) return fail(MHFD_ERR_INVALID_ARG, "null workspace (this plan needs %zu bytes)", need);
        if (reinterpret_cast<uintptr_t>(d_ws) % 4)
            return fail(MHFD_ERR_INVALID_ARG, "workspace not 4-byte aligned");
        if (ws_bytes < need)
            return fail(MHFD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    }
    if ((st = check_device(p)) != MHFD_OK) return st;
    return enqueue_log_stack(p, d_img, h, w, pitch, d_stack, static_cast<uint32_t*>(d_ws),
                             static_cast<hipStream_t>(stream));
}

mhfd_status mhfd_log_stack_static(mhfd_plan p, const void* d_img, int32_t h, int32_t w,
                                  int64_t pitch, float* d_stack, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_img, h, w, pitch);
    if (st != MHFD_OK) return st;
    if (!d_stack) return fail(MHFD_ERR_INVALID_ARG, "null stack");
    const size_t need = log_stack_scratch(p, h, w);
    if (need > MHFD_STATIC_SCRATCH_BYTES)
        return fail(MHFD_ERR_UNSUPPORTED, "the plan needs %zu bytes of scratch, the static array "
                    "holds %d", need, MHFD_STATIC_SCRATCH_BYTES);
    if ((st = check_device(p)) != MHFD_OK) return st;
    if (!p->d_scratch) return fail(MHFD_ERR_HIP, "no static scratch on device %d", p->device);
    return enqueue_log_stack(p, d_img, h, w, pitch, d_stack, p->d_scratch,
                             static_cast<hipStream_t>(stream));
}

mhfd_status mhfd_stretch_levels(const uint8_t* d_img, int32_t h, int32_t w, int64_t pitch,
                                int32_t* d_hist, int32_t* d_levels, void* stream) {
    g_last_error.clear();
    if (!d_img || !d_hist || !d_levels) return fail(MHFD_ERR_INVALID_ARG, "null pointer argument");
    if (h < 1 || w < 1 || pitch < w)
        return fail(MHFD_ERR_INVALID_ARG, "image %d x %d with pitch %lld", h, w,
                    static_cast<long long>(pitch));
    if (static_cast<int64_t>(h) * w > (int64_t(1) << 31) - 1)
        return fail(MHFD_ERR_UNSUPPORTED, "image above 2^31 - 1 pixels");
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = mhfd::launch_stretch_levels(d_img, h, w, pitch, d_hist, 1, nullptr, d_levels, n_cu,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "histogram stretch levels");
    return MHFD_OK;
}

mhfd_status mhfd_detect_stack(mhfd_plan p, const float* d_stack, int32_t h, int32_t w,
                              mhfd_blob* d_blobs, int32_t capacity, mhfd_result* d_result,
                              void* d_ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_stack, h, w, w);
    if (st != MHFD_OK) return st;
    DetectLayout L;
    if ((st = check_outputs(p, h, w, d_blobs, capacity, d_result, d_ws, ws_bytes, &L)) != MHFD_OK)
        return st;
    if ((st = check_device(p)) != MHFD_OK) return st;
    return enqueue_tail(p, d_stack, h, w, L, static_cast<char*>(d_ws), d_blobs, capacity, d_result,
                        static_cast<hipStream_t>(stream));
}

size_t mhfd_activity_bytes(mhfd_plan p, int32_t h, int32_t w) {
    if (!p || h < 1 || w < 1 || h > p->max_h || w > p->max_w || !sparse_stack(p)) return 0;
    return sizeof(uint64_t) * static_cast<size_t>(p->K) * ((h + 15) / 16) * ((w + 15) / 16);
}

mhfd_status mhfd_log_stack_sparse(mhfd_plan p, const void* d_img, int32_t h, int32_t w,
                                  int64_t pitch, float* d_stack, uint64_t* d_act, void* d_ws,
                                  size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_img, h, w, pitch);
    if (st != MHFD_OK) return st;
    if (!sparse_stack(p))
        return fail(MHFD_ERR_UNSUPPORTED, "this plan has no threshold-sparse stack (DoG criterion "
                    "or a radius above 56)");
    if (!d_stack || !d_act) return fail(MHFD_ERR_INVALID_ARG, "null stack or activity words");
    if (reinterpret_cast<uintptr_t>(d_act) % 8)
        return fail(MHFD_ERR_INVALID_ARG, "activity words not 8-byte aligned");
    const size_t need = log_stack_scratch(p, h, w);
    if (need) {
        if (!d_ws) return fail(MHFD_ERR_INVALID_ARG, "null workspace (this plan needs %zu bytes)", need);
        if (reinterpret_cast<uintptr_t>(d_ws) % 4)
            return fail(MHFD_ERR_INVALID_ARG, "workspace not 4-byte aligned");
        if (ws_bytes < need)
            return fail(MHFD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    }
    if ((st = check_device(p)) != MHFD_OK) return st;
    const mhfd::ActOut act{d_act, (w + 15) / 16, (h + 15) / 16, p->threshold};
    return enqueue_log_stack(p, d_img, h, w, pitch, d_stack, static_cast<uint32_t*>(d_ws),
                             static_cast<hipStream_t>(stream), act);
}

mhfd_status mhfd_detect_stack_sparse(mhfd_plan p, const float* d_stack, const uint64_t* d_act,
                                     int32_t h, int32_t w, mhfd_blob* d_blobs, int32_t capacity,
                                     mhfd_result* d_result, void* d_ws, size_t ws_bytes,
                                     void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_stack, h, w, w);
    if (st != MHFD_OK) return st;
    if (!sparse_stack(p))
        return fail(MHFD_ERR_UNSUPPORTED, "this plan has no threshold-sparse stack (DoG criterion "
                    "or a radius above 56)");
    if (!d_act || reinterpret_cast<uintptr_t>(d_act) % 8)
        return fail(MHFD_ERR_INVALID_ARG, "null or misaligned activity words");
    DetectLayout L;
    if ((st = check_outputs(p, h, w, d_blobs, capacity, d_result, d_ws, ws_bytes, &L)) != MHFD_OK)
        return st;
    if ((st = check_device(p)) != MHFD_OK) return st;
    return enqueue_tail(p, d_stack, h, w, L, static_cast<char*>(d_ws), d_blobs, capacity, d_result,
                        static_cast<hipStream_t>(stream), d_act);
}

mhfd_status mhfd_detect(mhfd_plan p, const void* d_img, int32_t h, int32_t w, int64_t pitch,
                        mhfd_blob* d_blobs, int32_t capacity, mhfd_result* d_result,
                        float* d_stack, void* d_ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_image(p, d_img, h, w, pitch);
    if (st != MHFD_OK) return st;
    DetectLayout L;
    if ((st = check_outputs(p, h, w, d_blobs, capacity, d_result, d_ws, ws_bytes, &L)) != MHFD_OK)
        return st;
    if ((st = check_device(p)) != MHFD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(d_ws);
    float* stack = d_stack ? d_stack : reinterpret_cast<float*>(base + L.stack);
    // Without a caller stack, only the part of the stack above the threshold
    // is written and read (the rest cannot change a decision).
    const bool sparse = !d_stack && L.act_bx > 0;
    const mhfd::ActOut act{sparse ? reinterpret_cast<uint64_t*>(base + L.act) : nullptr,
                           L.act_bx, L.act_by, p->threshold};
    if ((st = enqueue_log_stack(p, d_img, h, w, pitch, stack,
                                reinterpret_cast<uint32_t*>(base + L.maxbits), s, act)) != MHFD_OK)
        return st;
    return enqueue_tail(p, stack, h, w, L, base, d_blobs, capacity, d_result, s, act.mask);
}

size_t mhfd_batch_workspace_size(mhfd_plan p, int32_t max_tiles, int64_t max_pixels) {
    BatchLayout L;
    if (!p || !batch_layout(p, max_tiles, max_pixels, &L)) return 0;
    return L.total;
}

mhfd_status mhfd_detect_batched(mhfd_plan p, int32_t n, const mhfd_tile* d_tiles,
                                int64_t max_pixels, const mhfd_batch_opts* opts, void* d_ws,
                                size_t ws_bytes, void* stream) {
    g_last_error.clear();
    if (!p) return fail(MHFD_ERR_INVALID_ARG, "null plan");
    const int log_per_cu = opts && opts->log_groups_per_cu ? opts->log_groups_per_cu : 2;
    const int nms_per_cu = opts && opts->nms_groups_per_cu ? opts->nms_groups_per_cu : 8;
    if (log_per_cu < 1 || log_per_cu > 8 || nms_per_cu < 1 || nms_per_cu > 32)
        return fail(MHFD_ERR_INVALID_ARG, "batch options out of range (log %d of 1..8, maxima %d "
                    "of 1..32 workgroups per compute unit)", log_per_cu, nms_per_cu);
    if (p->stretch || p->criterion != MHFD_CRITERION_LOG || p->blur != MHFD_BLUR_DIRECT)
        return fail(MHFD_ERR_UNSUPPORTED, "batched detection takes plain LoG plans only");
    if (!d_tiles || !d_ws) return fail(MHFD_ERR_INVALID_ARG, "null tiles or workspace");
    BatchLayout L;
    if (!batch_layout(p, n, max_pixels, &L))
        return fail(MHFD_ERR_INVALID_ARG, "batch of %d tiles / %lld pixels outside [1, %d] / [1, 2^31)",
                    n, (long long)max_pixels, MHFD_MAX_BATCH);
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(MHFD_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    if (ws_bytes < L.total)
        return fail(MHFD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.total);
    mhfd_status st = check_device(p);
    if (st != MHFD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(d_ws);
    float* stack = reinterpret_cast<float*>(base + L.stack);
    // threshold-sparse stacks when the plan allows them (as mhfd_detect
    // without a caller stack)
    uint64_t* act = sparse_stack(p) ? reinterpret_cast<uint64_t*>(base + L.act) : nullptr;
    auto* tiles = reinterpret_cast<mhfd::BatchTile*>(base + L.tiles);
    auto* ctr = reinterpret_cast<mhfd::BatchCounters*>(base + L.ctr);
    hipError_t e = mhfd::launch_batch_setup(d_tiles, n, max_pixels, p->K, p->max_h, p->max_w,
                                            p->dtype, p->d_frags ? 1 : 0, tiles, ctr, s);
    if (e != hipSuccess) return hip_fail(e, "batch setup");
    // Matrix-core scales, one persistent launch per shape, the
    // costliest shape first; the same per-wave arithmetic as the single-tile
    // path, so every tile's stack equals its single-tile stack.
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(base + L.maxbits);
    const auto shapes = mfma_shapes(p);
    if (!shapes.empty() && p->dtype == MHFD_F32) {
        e = mhfd::launch_absmax_batch(n, tiles, ctr, maxbits, 8 * p->n_cu, s);
        if (e != hipSuccess) return hip_fail(e, "batched input range pass");
    }
    for (const auto& key : shapes) {
        mhfd::MfmaBatchScales sc{};
        for (int k = 0; k < p->K; ++k) {
            if (p->mfma_off[k] < 0) continue;
            const mhfd::MfmaShape m = mhfd::mfma_shape(p->radii[k]);
            if (m.nkr != key.first || m.nkc != key.second) continue;
            sc.rw8[sc.n] = m.rw8;
            sc.rwc[sc.n] = m.rwc;
            sc.frag_off[sc.n] = p->mfma_off[k];
            sc.plane[sc.n] = k;
            sc.out_scale[sc.n] = p->mfma_out_scale[k];
            ++sc.n;
        }
        const int slot = mfma_slot(key);
        if (slot < 0 || slot >= mhfd::MFMA_SHAPES)
            return fail(MHFD_ERR_UNSUPPORTED, "no matrix-core counter for shape %d x %d",
                        key.first, key.second);
        e = mhfd::launch_log_mfma_batch(p->dtype, key.first, key.second, n, tiles,
                                        p->dtype == MHFD_F32 ? maxbits : nullptr, stack,
                                        p->d_frags, sc, ctr, slot, log_per_cu * p->n_cu, act,
                                        p->threshold, s);
        if (e != hipSuccess) return hip_fail(e, "batched LoG (matrix cores) launch");
    }
    for (int cls = 2; cls >= 0; --cls) {
        mhfd::BatchScales sc{};
        std::vector<int> ks;
        for (int k = 0; k < p->K; ++k)
            if (mhfd::log_radius_class(p->padded[k]) == cls &&
                (p->mfma_off.empty() || p->mfma_off[k] < 0))
                ks.push_back(k);
        std::sort(ks.begin(), ks.end(), [&](int a, int b) {
            return p->padded[a] != p->padded[b] ? p->padded[a] > p->padded[b] : a < b;
        });
        for (int k : ks) {
            sc.radius[sc.n] = p->padded[k];
            sc.tap_off[sc.n] = p->tap_off[k];
            sc.plane[sc.n] = k;
            ++sc.n;
        }
        if (!sc.n) continue;
        e = mhfd::launch_log_batch(cls, p->dtype, n, tiles, p->K, stack, p->d_taps, sc, ctr,
                                   log_per_cu * p->n_cu, s);
        if (e != hipSuccess) return hip_fail(e, "batched LoG launch");
    }
    mhfd::BatchLaunchArgs a{};
    a.K = p->K;
    a.n_tiles = n;
    a.n_blk_bound = L.n_blk_bound;
    a.nms_grid = nms_per_cu * p->n_cu;
    a.reach = p->reach;
    a.d2top = p->d2_top;
    a.tau = p->threshold;
    a.cap = L.cap;
    a.stack = stack;
    a.act = act;
    a.tiles = tiles;
    a.blk_n = reinterpret_cast<int32_t*>(base + L.blk_n);
    a.blk_o = reinterpret_cast<int32_t*>(base + L.blk_o);
    a.blk_off = reinterpret_cast<int32_t*>(base + L.blk_off);
    a.keep = reinterpret_cast<int32_t*>(base + L.keep);
    a.keep_off = reinterpret_cast<int32_t*>(base + L.keep_off);
    a.scan_sums = reinterpret_cast<int32_t*>(base + L.scan_sums);
    a.pool = reinterpret_cast<mhfd::Cand*>(base + L.pool);
    a.cand = reinterpret_cast<mhfd::Cand*>(base + L.cand);
    a.d2max = p->d_d2max;
    a.sigmas = p->d_sigmas;
    a.ctr = ctr;
    e = mhfd::launch_batch_tail(a, s);
    if (e != hipSuccess) return hip_fail(e, "batched detection launch");
    return MHFD_OK;
}

size_t mhfd_focus_workspace_size(mhfd_plan p, int32_t b, int32_t h, int32_t w) {
    if (!p || b < 1 || h < 1 || w < 1 || h > p->max_h || w > p->max_w) return 0;
    return focus_layout(p, b, h, w).total;
}

mhfd_status mhfd_focus_score(mhfd_plan p, const float* d_imgs, int32_t b, int32_t h, int32_t w,
                             const float* d_sigmas, float beta, float tau, float* d_scores,
                             int32_t* d_error, void* d_ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_focus(p, d_imgs, b, h, w, d_sigmas, beta, tau, d_ws, ws_bytes);
    if (st != MHFD_OK) return st;
    if (!d_scores) return fail(MHFD_ERR_INVALID_ARG, "null score buffer");
    if ((st = check_device(p)) != MHFD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FocusLayout F = focus_layout(p, b, h, w);
    char* base = static_cast<char*>(d_ws);
    float* taps = reinterpret_cast<float*>(base + F.taps);
    double* partial = reinterpret_cast<double*>(base + F.partial);
    hipError_t e = mhfd::launch_soft_taps(d_sigmas, F.lay, taps, d_error, s);
    if (e != hipSuccess) return hip_fail(e, "soft tap synthesis");
    const std::vector<int>& P = p->focus_padded;
    mhfd::SoftPartials sp{};
    long long done = 0;
    if (F.mfma) {
        uint16_t* frags = reinterpret_cast<uint16_t*>(base + F.frags);
        float* scales = reinterpret_cast<float*>(base + F.scales);
        uint32_t* maxbits = reinterpret_cast<uint32_t*>(base + F.maxbits);
        if ((e = mhfd::launch_soft_frags(taps, F.lay, F.fl, frags, scales, s)) != hipSuccess ||
            (e = mhfd::launch_absmax_images(d_imgs, b, h, w, maxbits, s)) != hipSuccess)
            return hip_fail(e, "soft score set-up");
        for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, all_scales(p), mhfd::SOFT_FWD)) {
            mhfd::MfmaLaunch L = ml.second;
            L.dev_scale = scales;
            L.partial = partial + done;
            L.beta = beta;
            L.tau = tau;
            e = mhfd::launch_log_mfma_soft(mhfd::EPI_SOFTSUM, ml.first, ml.first, d_imgs, h, w, b,
                                           maxbits, frags, L, nullptr, s);
            if (e != hipSuccess) return hip_fail(e, "soft score launch");
            const int per_image = mfma_launch_blocks(L) * mhfd::mfma_waves_per_block();
            sp.base[sp.n] = done;
            sp.blocks[sp.n] = per_image;
            ++sp.n;
            done += static_cast<long long>(per_image) * b;
        }
        e = mhfd::launch_soft_finish(partial, sp, b, 1.0 / (static_cast<double>(p->K) * h * w),
                                     d_scores, s);
        if (e != hipSuccess) return hip_fail(e, "soft score finish");
        return MHFD_OK;
    }
    auto launches = make_launches(
        p, h, w, all_scales(p),
        [&](int k) { return F.lay.offset[k] + mhfd::SOFT_FWD * 4 * (P[k] + 1); },
        [](int k) { return k; }, [&](int k) { return P[k]; });
    for (auto& cl : launches) {
        mhfd::StackIO io{};
        io.img_batch = static_cast<long long>(h) * w;
        io.partial = partial + done;
        io.total_blocks = launch_blocks(cl.second);
        io.beta = beta;
        io.tau = tau;
        e = mhfd::launch_log_class(cl.first, MHFD_F32, mhfd::EPI_SOFTSUM, d_imgs, h, w, w, b, taps,
                                   cl.second, io, s);
        if (e != hipSuccess) return hip_fail(e, "soft score launch");
        sp.base[sp.n] = done;
        sp.blocks[sp.n] = io.total_blocks;
        ++sp.n;
        done += static_cast<long long>(io.total_blocks) * b;
    }
    e = mhfd::launch_soft_finish(partial, sp, b, 1.0 / (static_cast<double>(p->K) * h * w),
                                 d_scores, s);
    if (e != hipSuccess) return hip_fail(e, "soft score finish");
    return MHFD_OK;
}

mhfd_status mhfd_focus_score_backward(mhfd_plan p, const float* d_imgs, int32_t b, int32_t h,
                                      int32_t w, const float* d_sigmas, float beta, float tau,
                                      const float* d_grad_scores, float* d_grad_imgs,
                                      float* d_grad_sigmas, int32_t* d_error, void* d_ws,
                                      size_t ws_bytes, void* stream) {
    g_last_error.clear();
    mhfd_status st = check_focus(p, d_imgs, b, h, w, d_sigmas, beta, tau, d_ws, ws_bytes);
    if (st != MHFD_OK) return st;
    if (!d_grad_scores || !d_grad_imgs || !d_grad_sigmas)
        return fail(MHFD_ERR_INVALID_ARG, "null gradient buffer");
    if ((st = check_device(p)) != MHFD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FocusLayout F = focus_layout(p, b, h, w);
    char* base = static_cast<char*>(d_ws);
    float* taps = reinterpret_cast<float*>(base + F.taps);
    float* rpl = reinterpret_cast<float*>(base + F.rplane);
    float* dpl = reinterpret_cast<float*>(base + F.dplane);
    double* cot = reinterpret_cast<double*>(base + F.cot);
    hipError_t e = mhfd::launch_soft_taps(d_sigmas, F.lay, taps, d_error, s);
    const std::vector<int>& P = p->focus_padded;
    if (e != hipSuccess) return hip_fail(e, "soft tap synthesis");
    const long long npix = static_cast<long long>(h) * w;
    const double inv_khw = 1.0 / (static_cast<double>(p->K) * h * w);
    const int ncb = F.cot_stride;
    uint16_t* frags = reinterpret_cast<uint16_t*>(base + F.frags);
    float* scales = reinterpret_cast<float*>(base + F.scales);
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(base + F.maxbits);
    if (F.mfma) {
        // the partial slots a scale's launch does not reach stay zero
        if ((e = mhfd::launch_soft_frags(taps, F.lay, F.fl, frags, scales, s)) != hipSuccess ||
            (e = mhfd::launch_absmax_images(d_imgs, b, h, w, maxbits, s)) != hipSuccess ||
            (e = mhfd::launch_zero_f64(cot, static_cast<long long>(p->K) * ncb, s)) != hipSuccess)
            return hip_fail(e, "soft score backward set-up");
    }
    for (int k = 0; k < p->K; ++k) {
        const std::vector<int> one{k};
        auto run = [&](int set, int epi, const float* src, float* dst) -> hipError_t {
            if (F.mfma) {  // src: the images, or the cotangent planes (range words b .. 2b-1)
                const uint32_t* range = src == d_imgs ? maxbits : maxbits + b;
                for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, one, set)) {
                    mhfd::MfmaLaunch L = ml.second;
                    L.dev_scale = scales;
                    hipError_t err = mhfd::launch_log_mfma_soft(epi, ml.first, ml.first, src, h, w,
                                                                b, range, frags, L, dst, s);
                    if (err != hipSuccess) return err;
                }
                return hipSuccess;
            }
            auto launches = make_launches(
                p, h, w, one, [&](int kk) { return F.lay.offset[kk] + set * 4 * (P[kk] + 1); },
                [](int) { return 0; }, [&](int kk) { return P[kk]; });
            mhfd::StackIO io{};
            io.img_batch = npix;
            io.out = dst;
            io.out_batch = npix;
            io.plane_stride = 0;
            for (auto& cl : launches) {
                hipError_t err = mhfd::launch_log_class(cl.first, MHFD_F32, epi, src, h, w, w, b,
                                                        taps, cl.second, io, s);
                if (err != hipSuccess) return err;
            }
            return hipSuccess;
        };
        // r = sigma^2 Lap I, d = D1 I + D2 I (the sigma-derivative of Lap I)
        if (F.mfma) {
            // r and D1 from one row pass (same row taps g, h)
            for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, one, mhfd::SOFT_FWD,
                                               mhfd::SOFT_D1)) {
                mhfd::MfmaLaunch L = ml.second;
                L.dev_scale = scales;
                L.aux = dpl;
                e = mhfd::launch_log_mfma_soft(mhfd::EPI_DUAL, ml.first, ml.first, d_imgs, h, w,
                                               b, maxbits, frags, L, rpl, s);
                if (e != hipSuccess) return hip_fail(e, "soft score backward recompute");
            }
        } else if ((e = run(mhfd::SOFT_FWD, mhfd::EPI_STORE, d_imgs, rpl)) != hipSuccess ||
                   (e = run(mhfd::SOFT_D1, mhfd::EPI_STORE, d_imgs, dpl)) != hipSuccess) {
            return hip_fail(e, "soft score backward recompute");
        }
        if (F.mfma) {
            // D2 on the matrix cores with the cotangent as its epilogue: r <- c
            // in place, sigma partials, max |c| per image for the adjoint
            for (auto& ml : soft_mfma_launches(p, F.fl, b, h, w, one, mhfd::SOFT_D2)) {
                mhfd::MfmaLaunch L = ml.second;
                L.dev_scale = scales;
                L.partial = cot + static_cast<long long>(k) * ncb;
                L.beta = beta;
                L.tau = tau;
                L.aux = rpl;
                L.sigmas = d_sigmas;
                L.soft_k = k;
                L.gbar = d_grad_scores;
                L.inv_khw = inv_khw;
                L.cmax = maxbits + b;
                e = mhfd::launch_log_mfma_soft(mhfd::EPI_COTAN, ml.first, ml.first, d_imgs, h, w,
                                               b, maxbits, frags, L, dpl, s);
                if (e != hipSuccess) return hip_fail(e, "soft score cotangent");
            }
        } else {
            if ((e = run(mhfd::SOFT_D2, mhfd::EPI_ACCUM, d_imgs, dpl)) != hipSuccess)
                return hip_fail(e, "soft score backward recompute");
            e = mhfd::launch_soft_cotangent(rpl, dpl, npix, b, d_sigmas, k, d_grad_scores,
                                            inv_khw, beta, tau,
                                            cot + static_cast<long long>(k) * ncb, nullptr, s);
            if (e != hipSuccess) return hip_fail(e, "soft score cotangent");
        }
        // dI (+)= Lap^T c = Lap c
        if ((e = run(mhfd::SOFT_ADJ, k == 0 ? mhfd::EPI_STORE : mhfd::EPI_ACCUM, rpl,
                     d_grad_imgs)) != hipSuccess)
            return hip_fail(e, "soft score adjoint");
    }
    e = mhfd::launch_sigma_grad_finish(cot, ncb, p->K, d_grad_sigmas, s);
    if (e != hipSuccess) return hip_fail(e, "sigma gradient finish");
    return MHFD_OK;
}

}  // extern "C"
