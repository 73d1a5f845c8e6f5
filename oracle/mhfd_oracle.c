/*
 * mhfd_oracle.c -- plain FP64 CPU oracle for the scale-normalised
 * Laplacian-of-Gaussian blob detector of "Ultrafast Focus Detection for
 * Automated Microscopy" (Multi-scale Histologic Feature Detection, MHFD).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the detector computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * library never links, loads or calls it, and it shares no code, header,
 * table or constant with the HIP path.
 *
 * Everything is double precision, row-major, with explicit loops.  OpenMP is
 * used only over independent outputs (rows, columns, records), and every
 * reduction is finished sequentially, so results do not depend on the thread
 * count.
 *
 * Readings of the paper that this file fixes (each one is listed with its
 * reason in the design notes of the repository):
 *   - scale t is the Gaussian standard deviation (section 2.2: the filter
 *     variance is t^2), and the detector response is the scale-normalised
 *     Laplacian  R_k = s * sigma_k^2 * Lap(G_sigma_k * I)  (section 2.2,
 *     equation "blobdetector" and the DoG approximation of t^2 Lap L that
 *     follows it), with s = -1 for bright blobs on a dark background;
 *   - kernels are the sampled Gaussian of section 2.2, truncated to the
 *     square support |i|,|j| <= R = floor(truncate*sigma + 0.5) and
 *     normalised to unit sum; the second-derivative taps use the discrete
 *     variance V of the truncated kernel,  h_j = (j^2 - V) g_j / sigma^4,
 *     which is exactly 2 dg_j/d(sigma^2) (heat-equation form of the scale
 *     derivative) and sums to zero, so a constant image has zero response;
 *   - borders use half-sample symmetric extension (... x1 x0 | x0 x1 ...);
 *   - a candidate is a voxel that equals the maximum of its 3x3x3
 *     scale-space window (the 3x3 maxpool-equality test of section 3,
 *     generalised from "local in space, global in scale" to local in both)
 *     and whose response is strictly above the threshold;
 *   - overlap pruning is one-shot dominance with blob radius sqrt(2)*sigma;
 *   - the histogram stretch of section 3 (Algorithm 1, first step) on 8-bit
 *     images saturates the darkest and the lightest 0.175% of the pixels:
 *     with q = 0.00175 N, the low level is the smallest code v with at
 *     least q pixels <= v and the high level the largest code with at least
 *     q pixels >= v; codes map to clip((v - low) / (high - low), 0, 1), and
 *     to 0 when high = low.  Counts are compared with q exactly, in
 *     integers: count >= 0.00175 N  <=>  100000 count >= 175 N;
 *   - the paper's own criterion (equation "dog" of section 2.2, equation
 *     "argmax" and Algorithm 1 of section 3): Gaussian planes
 *     L_i = G_{t_i} * I on the same sampled, truncated, reflected kernels;
 *     DoG_i = t_i (L_{i+1} - L_i) for i < K - 1; per pixel the largest DoG
 *     over scale (the first scale on ties, as an argmax gives); a pixel
 *     counts when that value equals the
 *     maximum of its 3x3 neighbourhood (maxpool equality, windows clipped
 *     at the image border) and exceeds the threshold.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_SQRT2 1.41421356237309504880

/* Kernel radius: the Gaussian is truncated at `truncate` standard deviations. */
int ora_radius(double sigma, double truncate)
{
    return (int)floor(truncate * sigma + 0.5);
}

/*
 * Gaussian and second-derivative taps for offsets j = -R..R (stored at j+R).
 * g_j = exp(-j^2 / (2 sigma^2)) / Z  -- the Gaussian of section 2.2, sampled
 *        at integers and normalised over the truncated support;
 * V   = sum_j j^2 g_j                 -- variance of the truncated kernel;
 * h_j = (j^2 - V) g_j / sigma^4       -- discrete d^2/dx^2 of the Gaussian.
 */
void ora_taps(double sigma, int R, double *g, double *h)
{
    double Z = 0.0, V = 0.0;
    for (int j = -R; j <= R; ++j) {
        double e = exp(-(double)j * (double)j / (2.0 * sigma * sigma));
        g[j + R] = e;
        Z += e;
    }
    for (int j = -R; j <= R; ++j)
        g[j + R] /= Z;
    for (int j = -R; j <= R; ++j)
        V += (double)j * (double)j * g[j + R];
    double s4 = sigma * sigma * sigma * sigma;
    for (int j = -R; j <= R; ++j)
        h[j + R] = ((double)j * (double)j - V) * g[j + R] / s4;
}

/*
 * sigma-derivatives of the taps above (radius held fixed):
 *   dg_j/dsigma = g_j (j^2 - V) / sigma^3
 *   dV/dsigma   = (M4 - V^2) / sigma^3,       M4 = sum_j j^4 g_j
 *   dh_j/dsigma = [(j^2 - V) dg_j - dV g_j] / sigma^4 - 4 (j^2 - V) g_j / sigma^5
 */
void ora_dtaps(double sigma, int R, double *gd, double *hd)
{
    int n = 2 * R + 1;
    double *g = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * n);
    ora_taps(sigma, R, g, h);
    double V = 0.0, M4 = 0.0;
    for (int j = -R; j <= R; ++j) {
        double j2 = (double)j * (double)j;
        V += j2 * g[j + R];
        M4 += j2 * j2 * g[j + R];
    }
    double s3 = sigma * sigma * sigma, s4 = s3 * sigma, s5 = s4 * sigma;
    double Vd = (M4 - V * V) / s3;
    for (int j = -R; j <= R; ++j) {
        double q = (double)j * (double)j - V;
        gd[j + R] = g[j + R] * q / s3;
        hd[j + R] = (q * gd[j + R] - Vd * g[j + R]) / s4 - 4.0 * q * g[j + R] / s5;
    }
    free(g);
    free(h);
}

/* Half-sample symmetric extension: index u of the infinite periodic
 * mirror (period 2n) of a line of n samples. */
long ora_ext(long u, long n)
{
    long m = u % (2 * n);
    if (m < 0)
        m += 2 * n;
    return m < n ? m : 2 * n - 1 - m;
}

/* out[y][x] = sum_j w_j in[y][ext(x - j)], j = -R..R  (1-D pass along x). */
static void pass_x(const double *in, int H, int W, const double *w, int R, double *out)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = -R; j <= R; ++j)
                acc += w[j + R] * in[(size_t)y * W + ora_ext((long)x - j, W)];
            out[(size_t)y * W + x] = acc;
        }
}

/* out[y][x] = sum_i w_i in[ext(y - i)][x], i = -R..R  (1-D pass along y). */
static void pass_y(const double *in, int H, int W, const double *w, int R, double *out)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int i = -R; i <= R; ++i)
                acc += w[i + R] * in[(size_t)ora_ext((long)y - i, H) * W + x];
            out[(size_t)y * W + x] = acc;
        }
}

/*
 * Laplacian of the Gaussian-smoothed image at one scale, separable form:
 *   A = g (*)_x I,  B = h (*)_x I,  Lap = h (*)_y A + g (*)_y B.
 * The 2-D Gaussian of section 2.2 is the product g(x) g(y), so its Laplacian
 * is h(x) g(y) + g(x) h(y); this is that kernel applied axis by axis.
 */
static void lap_separable(const double *img, int H, int W, double sigma, int R, double *lap)
{
    int n = 2 * R + 1;
    size_t N = (size_t)H * W;
    double *g = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * n);
    double *A = (double *)malloc(sizeof(double) * N);
    double *B = (double *)malloc(sizeof(double) * N);
    double *T = (double *)malloc(sizeof(double) * N);
    ora_taps(sigma, R, g, h);
    pass_x(img, H, W, g, R, A);
    pass_x(img, H, W, h, R, B);
    pass_y(A, H, W, h, R, lap);
    pass_y(B, H, W, g, R, T);
    for (size_t p = 0; p < N; ++p)
        lap[p] += T[p];
    free(g); free(h); free(A); free(B); free(T);
}

/*
 * Scale-normalised LoG stack: out[k][y][x] = s * sigma_k^2 * Lap_k[y][x],
 * s = -1 when polarity == 0 (bright blobs), +1 when polarity == 1.
 */
void ora_log_stack(const double *img, int H, int W, int K, const double *sigmas,
                   double truncate, int polarity, double *out)
{
    double s = polarity == 0 ? -1.0 : 1.0;
    size_t N = (size_t)H * W;
    for (int k = 0; k < K; ++k) {
        double sg = sigmas[k];
        int R = ora_radius(sg, truncate);
        double *plane = out + (size_t)k * N;
        lap_separable(img, H, W, sg, R, plane);
        for (size_t p = 0; p < N; ++p)
            plane[p] *= s * sg * sg;
    }
}

/*
 * One voxel of the same stack from the plain 2-D definition: a direct sum
 * over the square support with the 2-D kernel h_i g_j + g_i h_j.
 */
double ora_log_point(const double *img, int H, int W, double sigma, double truncate,
                     int polarity, int y, int x)
{
    int R = ora_radius(sigma, truncate);
    int n = 2 * R + 1;
    double *g = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * n);
    ora_taps(sigma, R, g, h);
    double acc = 0.0;
    for (int i = -R; i <= R; ++i) {
        long yy = ora_ext((long)y - i, H);
        for (int j = -R; j <= R; ++j) {
            long xx = ora_ext((long)x - j, W);
            acc += (h[i + R] * g[j + R] + g[i + R] * h[j + R]) * img[(size_t)yy * W + xx];
        }
    }
    free(g);
    free(h);
    double s = polarity == 0 ? -1.0 : 1.0;
    return s * sigma * sigma * acc;
}

/* Whole stack from the 2-D definition (for tiny images only). */
void ora_log_direct(const double *img, int H, int W, int K, const double *sigmas,
                    double truncate, int polarity, double *out)
{
    for (int k = 0; k < K; ++k)
#pragma omp parallel for schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                out[((size_t)k * H + y) * W + x] =
                    ora_log_point(img, H, W, sigmas[k], truncate, polarity, y, x);
}

/* Maximum of the 3x3x3 window around (k, y, x), clipped to the volume.
 * If `skip_centre` the centre voxel is left out (-inf if nothing remains). */
static double window_max(const double *st, int K, int H, int W, int k, int y, int x, int skip_centre)
{
    double m = -INFINITY;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int kk = k + dk, yy = y + dy, xx = x + dx;
                if (kk < 0 || kk >= K || yy < 0 || yy >= H || xx < 0 || xx >= W)
                    continue;
                if (skip_centre && dk == 0 && dy == 0 && dx == 0)
                    continue;
                double v = st[((size_t)kk * H + yy) * W + xx];
                if (v > m)
                    m = v;
            }
    return m;
}

/*
 * Candidate blobs: voxels equal to the maximum of their 3x3x3 window whose
 * response is strictly greater than tau.  Records (y, x, k) are written in
 * ascending (y, x, k) order with their response; at most `cap` are written
 * and the true number is returned.
 */
long ora_candidates(const double *st, int K, int H, int W, double tau,
                    int32_t *ykx, double *resp, long cap)
{
    long n = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int k = 0; k < K; ++k) {
                double v = st[((size_t)k * H + y) * W + x];
                if (!(v > tau))
                    continue;
                if (v >= window_max(st, K, H, W, k, y, x, 0)) {
                    if (n < cap) {
                        ykx[3 * n + 0] = y;
                        ykx[3 * n + 1] = x;
                        ykx[3 * n + 2] = k;
                        resp[n] = v;
                    }
                    ++n;
                }
            }
    return n;
}

/*
 * Decision margin.  The candidate decision of a voxel is "ambiguous at eps"
 * when a perturbation of at most eps could flip it: the voxel could still be
 * a candidate (value >= tau - eps and >= m - eps, m the largest of its other
 * window neighbours) and it lies within eps of tau or within eps of m.  A
 * voxel that is clearly below a neighbour or clearly below tau decides
 * nothing, however close it is to either.  Returns the number of ambiguous
 * voxels and, if `mask` is non-null, marks them (K*H*W bytes).
 */
long ora_ambiguous(const double *st, int K, int H, int W, double tau, double eps, uint8_t *mask)
{
    long n = 0;
#pragma omp parallel for collapse(2) reduction(+ : n) schedule(static)
    for (int k = 0; k < K; ++k)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t p = ((size_t)k * H + y) * W + x;
                double v = st[p];
                double m = window_max(st, K, H, W, k, y, x, 1);
                int amb = 0;
                if (v >= tau - eps && v >= m - eps)
                    amb = fabs(v - tau) <= eps || fabs(v - m) <= eps;
                if (mask)
                    mask[p] = (uint8_t)amb;
                n += amb;
            }
    return n;
}

/*
 * Fraction of the smaller disc covered by the intersection of two discs
 * (centres a, b; radii ra, rb): 0 when disjoint, 1 when one contains the
 * other, otherwise the circular-lens area over pi * min(ra, rb)^2.
 */
double ora_overlap(double ya, double xa, double ra, double yb, double xb, double rb)
{
    double dy = ya - yb, dx = xa - xb;
    double d = sqrt(dy * dy + dx * dx);
    double rmin = ra < rb ? ra : rb;
    if (d >= ra + rb)
        return 0.0;
    if (d <= fabs(ra - rb))
        return 1.0;
    double c1 = (d * d + ra * ra - rb * rb) / (2.0 * d * ra);
    double c2 = (d * d + rb * rb - ra * ra) / (2.0 * d * rb);
    double area = ra * ra * acos(c1) + rb * rb * acos(c2)
                - 0.5 * sqrt((-d + ra + rb) * (d + ra - rb) * (d - ra + rb) * (d + ra + rb));
    return area / (M_PI * rmin * rmin);
}

/*
 * One-shot overlap pruning.  Blob a dominates b when it has the larger scale
 * index, or the same scale index and the lexicographically smaller (y, x).
 * b is removed iff some a != b in the input list dominates b and their
 * overlap exceeds theta.  Radius of a blob at scale sigma is sqrt(2) sigma.
 * ykx: n records (y, x, k); sig[k]: sigma of scale k.  keep[b] in {0, 1}.
 */
void ora_prune(const int32_t *ykx, const double *sig, long n, double theta, uint8_t *keep)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (long b = 0; b < n; ++b) {
        int yb = ykx[3 * b], xb = ykx[3 * b + 1], kb = ykx[3 * b + 2];
        double rb = ORA_SQRT2 * sig[kb];
        uint8_t kp = 1;
        for (long a = 0; a < n && kp; ++a) {
            if (a == b)
                continue;
            int ya = ykx[3 * a], xa = ykx[3 * a + 1], ka = ykx[3 * a + 2];
            int dom = ka > kb || (ka == kb && (ya < yb || (ya == yb && xa < xb)));
            if (!dom)
                continue;
            double ra = ORA_SQRT2 * sig[ka];
            if (ora_overlap(ya, xa, ra, yb, xb, rb) > theta)
                kp = 0;
        }
        keep[b] = kp;
    }
}

/* softplus(z) = log(1 + e^z), written so it neither overflows nor loses
 * the small-argument tail. */
static double softplus(double z)
{
    return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
}

static double sigmoid(double z)
{
    return 1.0 / (1.0 + exp(-z));
}

/*
 * Soft focus score, one value per image b:
 *   S_b = 1/(K H W) sum_k sum_{y,x} softplus(beta (|r_k[y,x]| - tau)),
 *   r_k = sigma_k^2 Lap_k  (the magnitude makes the polarity irrelevant).
 * radii[k] fixes the kernel radius of scale k.
 */
void ora_soft_score(const double *imgs, int Bn, int H, int W, int K, const double *sigmas,
                    const int *radii, double beta, double tau, double *scores)
{
    size_t N = (size_t)H * W;
    double *lap = (double *)malloc(sizeof(double) * N);
    double *rowsum = (double *)malloc(sizeof(double) * H);
    for (int b = 0; b < Bn; ++b) {
        double S = 0.0;
        for (int k = 0; k < K; ++k) {
            double sg = sigmas[k];
            lap_separable(imgs + (size_t)b * N, H, W, sg, radii[k], lap);
#pragma omp parallel for schedule(static)
            for (int y = 0; y < H; ++y) {
                double a = 0.0;
                for (int x = 0; x < W; ++x) {
                    double r = sg * sg * lap[(size_t)y * W + x];
                    a += softplus(beta * (fabs(r) - tau));
                }
                rowsum[y] = a;
            }
            for (int y = 0; y < H; ++y)
                S += rowsum[y];
        }
        scores[b] = S / ((double)K * (double)N);
    }
    free(lap);
    free(rowsum);
}

/* Adjoint of pass_y by explicit scatter through the border extension:
 * out[ext(y - i)][x] += w_i in[y][x]. */
static void pass_y_adjoint(const double *in, int H, int W, const double *w, int R, double *out)
{
    memset(out, 0, sizeof(double) * (size_t)H * W);
#pragma omp parallel for schedule(static)
    for (int x = 0; x < W; ++x)
        for (int y = 0; y < H; ++y) {
            double v = in[(size_t)y * W + x];
            for (int i = -R; i <= R; ++i)
                out[(size_t)ora_ext((long)y - i, H) * W + x] += w[i + R] * v;
        }
}

/* Adjoint of pass_x by explicit scatter: out[y][ext(x - j)] += w_j in[y][x]. */
static void pass_x_adjoint_acc(const double *in, int H, int W, const double *w, int R, double *out)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double v = in[(size_t)y * W + x];
            for (int j = -R; j <= R; ++j)
                out[(size_t)y * W + ora_ext((long)x - j, W)] += w[j + R] * v;
        }
}

/*
 * Gradient of the soft focus score for upstream gradients gbar[b]:
 *   w_k   = gbar_b/(K H W) * beta * sigmoid(beta (|r_k| - tau)) * sgn(r_k),
 *           with sgn(0) = 0;
 *   dI_b  = sum_k C_k^T (sigma_k^2 w_k), C_k = the Laplacian operator of
 *           lap_separable, applied transposed by explicit scatter;
 *   dsig_k = sum_b sum_{y,x} w_k * (2 sigma_k Lap_k + sigma_k^2 D_k),
 *           D_k = (h'(y) g(x) + h(y) g'(x) + g'(y) h(x) + g(y) h'(x)) (*) I,
 *           primes being the sigma-derivatives of ora_dtaps.
 * dimgs (B*H*W) and dsig (K) are overwritten.
 */
void ora_soft_score_grad(const double *imgs, int Bn, int H, int W, int K, const double *sigmas,
                         const int *radii, double beta, double tau, const double *gbar,
                         double *dimgs, double *dsig)
{
    size_t N = (size_t)H * W;
    double *A = (double *)malloc(sizeof(double) * N);
    double *Bp = (double *)malloc(sizeof(double) * N);
    double *Ad = (double *)malloc(sizeof(double) * N);
    double *Bd = (double *)malloc(sizeof(double) * N);
    double *lap = (double *)malloc(sizeof(double) * N);
    double *D = (double *)malloc(sizeof(double) * N);
    double *T = (double *)malloc(sizeof(double) * N);
    double *c = (double *)malloc(sizeof(double) * N);
    double *rowsum = (double *)malloc(sizeof(double) * H);
    memset(dimgs, 0, sizeof(double) * N * Bn);
    for (int k = 0; k < K; ++k)
        dsig[k] = 0.0;
    for (int k = 0; k < K; ++k) {
        double sg = sigmas[k];
        int R = radii[k], n = 2 * R + 1;
        double *g = (double *)malloc(sizeof(double) * n);
        double *h = (double *)malloc(sizeof(double) * n);
        double *gd = (double *)malloc(sizeof(double) * n);
        double *hd = (double *)malloc(sizeof(double) * n);
        ora_taps(sg, R, g, h);
        ora_dtaps(sg, R, gd, hd);
        for (int b = 0; b < Bn; ++b) {
            const double *I = imgs + (size_t)b * N;
            double scale = gbar[b] / ((double)K * (double)N);
            /* forward quantities */
            pass_x(I, H, W, g, R, A);
            pass_x(I, H, W, h, R, Bp);
            pass_x(I, H, W, gd, R, Ad);
            pass_x(I, H, W, hd, R, Bd);
            pass_y(A, H, W, h, R, lap);
            pass_y(Bp, H, W, g, R, T);
            for (size_t p = 0; p < N; ++p)
                lap[p] += T[p];
            /* D = hd (*)_y A + h (*)_y Ad + gd (*)_y B + g (*)_y Bd */
            pass_y(A, H, W, hd, R, D);
            pass_y(Ad, H, W, h, R, T);
            for (size_t p = 0; p < N; ++p) D[p] += T[p];
            pass_y(Bp, H, W, gd, R, T);
            for (size_t p = 0; p < N; ++p) D[p] += T[p];
            pass_y(Bd, H, W, g, R, T);
            for (size_t p = 0; p < N; ++p) D[p] += T[p];
            /* cotangent, sigma partials */
#pragma omp parallel for schedule(static)
            for (int y = 0; y < H; ++y) {
                double a = 0.0;
                for (int x = 0; x < W; ++x) {
                    size_t p = (size_t)y * W + x;
                    double r = sg * sg * lap[p];
                    double sgn = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);
                    double w = scale * beta * sigmoid(beta * (fabs(r) - tau)) * sgn;
                    a += w * (2.0 * sg * lap[p] + sg * sg * D[p]);
                    c[p] = w * sg * sg;
                }
                rowsum[y] = a;
            }
            for (int y = 0; y < H; ++y)
                dsig[k] += rowsum[y];
            /* image adjoint: C^T c = g_x^T h_y^T c + h_x^T g_y^T c */
            double *dI = dimgs + (size_t)b * N;
            pass_y_adjoint(c, H, W, h, R, T);
            pass_x_adjoint_acc(T, H, W, g, R, dI);
            pass_y_adjoint(c, H, W, g, R, T);
            pass_x_adjoint_acc(T, H, W, h, R, dI);
        }
        free(g); free(h); free(gd); free(hd);
    }
    free(A); free(Bp); free(Ad); free(Bd); free(lap); free(D); free(T); free(c); free(rowsum);
}

/*
 * Adjoint of the scale-normalised LoG at one scale applied to a field c,
 * by explicit scatter (no symmetry assumed): out = s sigma^2 C^T c.
 * Used to check that the operator is self-adjoint under the half-sample
 * extension.
 */
void ora_log_adjoint(const double *c, int H, int W, double sigma, double truncate,
                     int polarity, double *out)
{
    int R = ora_radius(sigma, truncate), n = 2 * R + 1;
    size_t N = (size_t)H * W;
    double *g = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * n);
    double *T = (double *)malloc(sizeof(double) * N);
    ora_taps(sigma, R, g, h);
    memset(out, 0, sizeof(double) * N);
    pass_y_adjoint(c, H, W, h, R, T);
    pass_x_adjoint_acc(T, H, W, g, R, out);
    pass_y_adjoint(c, H, W, g, R, T);
    pass_x_adjoint_acc(T, H, W, h, R, out);
    double s = polarity == 0 ? -1.0 : 1.0;
    for (size_t p = 0; p < N; ++p)
        out[p] *= s * sigma * sigma;
    free(g); free(h); free(T);
}

/* Histogram stretch levels of an 8-bit image (section 3; Algorithm 1, first
 * step), from the definition: the histogram is counted, then the low level
 * walks up from code 0 and the high level down from 255 until the running
 * count reaches q = 0.00175 N.  hist[256] receives the counts. */
void ora_stretch_levels(const uint8_t *img, int H, int W, long pitch, int64_t *hist,
                        int *low, int *high)
{
    const int64_t N = (int64_t)H * W;
    for (int v = 0; v < 256; ++v) hist[v] = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) hist[img[(long)y * pitch + x]] += 1;
    int64_t run = 0;
    int lo = 0;
    for (; lo < 255; ++lo) {
        run += hist[lo];
        if (100000 * run >= 175 * N) break;
    }
    run = 0;
    int hi = 255;
    for (; hi > 0; --hi) {
        run += hist[hi];
        if (100000 * run >= 175 * N) break;
    }
    *low = lo;
    *high = hi;
}

/* The stretched image in [0, 1] (FP64), H x W row-major. */
void ora_stretch(const uint8_t *img, int H, int W, long pitch, double *out, int *low, int *high)
{
    int64_t hist[256];
    ora_stretch_levels(img, H, W, pitch, hist, low, high);
    const int lo = *low, hi = *high;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int v = img[(long)y * pitch + x];
            double o = 0.0;
            if (hi > lo) {
                o = (double)(v - lo) / (double)(hi - lo);
                if (o < 0.0) o = 0.0;
                if (o > 1.0) o = 1.0;
            }
            out[(long)y * W + x] = o;
        }
}

/* Gaussian planes L_k = G_{sigma_k} * I (section 2.2), separable, reflected:
 * out[k][y][x]. */
void ora_gauss_stack(const double *img, int H, int W, int K, const double *sigmas,
                     double truncate, double *out)
{
    size_t N = (size_t)H * W;
    double *T = (double *)malloc(sizeof(double) * N);
    for (int k = 0; k < K; ++k) {
        int R = ora_radius(sigmas[k], truncate);
        double *g = (double *)malloc(sizeof(double) * (2 * R + 1));
        double *h = (double *)malloc(sizeof(double) * (2 * R + 1));
        ora_taps(sigmas[k], R, g, h);
        pass_x(img, H, W, g, R, T);
        pass_y(T, H, W, g, R, out + (size_t)k * N);
        free(g);
        free(h);
    }
    free(T);
}

/*
 * The paper's criterion on Gaussian planes L (K planes at scales t_k):
 * DoG_i = t_i (L_{i+1} - L_i), i = 0..K-2 (equation "dog"); M = max_i DoG_i
 * with idx = the first i attaining it (the inner argmax of equation
 * "argmax"); C = pixels with M > tau and M equal to the maximum of M over
 * their 3x3 neighbourhood, clipped at the border (the outer argmaxlocal as a
 * maxpool comparison).  M and idx are H x W outputs; up to `cap` records
 * (y, x, idx) are written in ascending (y, x) order; returns |C|.
 */
long ora_dog_criterion(const double *L, int H, int W, int K, const double *sigmas, double tau,
                       double *M, int32_t *idx, int32_t *yxk, long cap)
{
    size_t N = (size_t)H * W;
    for (size_t p = 0; p < N; ++p) {
        double best = -INFINITY;
        int bi = 0;
        for (int i = 0; i + 1 < K; ++i) {
            double d = sigmas[i] * (L[(size_t)(i + 1) * N + p] - L[(size_t)i * N + p]);
            if (d > best) {
                best = d;
                bi = i;
            }
        }
        M[p] = best;
        idx[p] = bi;
    }
    long n = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double v = M[(size_t)y * W + x];
            if (!(v > tau))
                continue;
            double m = -INFINITY;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    if (M[(size_t)yy * W + xx] > m)
                        m = M[(size_t)yy * W + xx];
                }
            if (v >= m) {
                if (n < cap) {
                    yxk[3 * n + 0] = y;
                    yxk[3 * n + 1] = x;
                    yxk[3 * n + 2] = idx[(size_t)y * W + x];
                }
                ++n;
            }
        }
    return n;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int ora_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = 1
#ifdef _OPENMP
            * omp_get_num_threads()
#endif
            ;
    }
    return n;
}

/* Set the number of OpenMP threads of the oracle's parallel loops (timing
 * of the single-thread baseline); n < 1 leaves it unchanged. */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
