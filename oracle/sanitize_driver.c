/* Test infrastructure: drives every entry point of the oracle (mhfd_oracle.c)
 * on small and degenerate inputs so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer sees each of its loops, borders and buffers:
 * one-pixel and one-row images, kernel radii far above the image size
 * (repeated reflection), candidate lists longer than their capacity, empty
 * prune lists, pitched 8-bit rows.  A few invariants are checked on the way
 * (a constant image has no LoG response; lists respect their capacity; the
 * overlap of a blob with itself is 1).  Prints "ok" and exits 0 when every
 * check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int ora_radius(double sigma, double truncate);
void ora_taps(double sigma, int R, double *g, double *h);
void ora_dtaps(double sigma, int R, double *gd, double *hd);
long ora_ext(long u, long n);
void ora_log_stack(const double *img, int H, int W, int K, const double *sigmas, double truncate,
                   int polarity, double *out);
double ora_log_point(const double *img, int H, int W, double sigma, double truncate,
                     int polarity, int y, int x);
void ora_log_direct(const double *img, int H, int W, int K, const double *sigmas,
                    double truncate, int polarity, double *out);
long ora_candidates(const double *st, int K, int H, int W, double tau, int32_t *ykx,
                    double *resp, long cap);
long ora_ambiguous(const double *st, int K, int H, int W, double tau, double eps, uint8_t *mask);
double ora_overlap(double ya, double xa, double ra, double yb, double xb, double rb);
void ora_prune(const int32_t *ykx, const double *sig, long n, double theta, uint8_t *keep);
void ora_soft_score(const double *imgs, int Bn, int H, int W, int K, const double *sigmas,
                    const int *radii, double beta, double tau, double *scores);
void ora_soft_score_grad(const double *imgs, int Bn, int H, int W, int K, const double *sigmas,
                         const int *radii, double beta, double tau, const double *gbar,
                         double *dimgs, double *dsig);
void ora_log_adjoint(const double *c, int H, int W, double sigma, double truncate, int polarity,
                     double *out);
void ora_stretch_levels(const uint8_t *img, int H, int W, long pitch, int64_t *hist, int *low,
                        int *high);
void ora_stretch(const uint8_t *img, int H, int W, long pitch, double *out, int *low, int *high);
void ora_gauss_stack(const double *img, int H, int W, int K, const double *sigmas,
                     double truncate, double *out);
long ora_dog_criterion(const double *L, int H, int W, int K, const double *sigmas, double tau,
                       double *M, int32_t *idx, int32_t *yxk, long cap);
int ora_threads(void);
void ora_set_threads(int n);

static int failures = 0;

static void check(int cond, const char *what)
{
    if (!cond) {
        printf("FAIL %s\n", what);
        ++failures;
    }
}

/* Deterministic pseudo-random values in [0, 1) (a 64-bit LCG). */
static double next_u(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static double *field(int n, uint64_t seed)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) a[i] = next_u(&seed);
    return a;
}

static void detector_case(int H, int W, int K, const double *sig, long cap)
{
    size_t N = (size_t)H * W;
    double *img = field((int)N, 17u + (uint64_t)H * 31u + (uint64_t)W);
    double *st = (double *)malloc(sizeof(double) * N * K);
    double *st2 = (double *)malloc(sizeof(double) * N * K);
    for (int pol = 0; pol < 2; ++pol) {
        ora_log_stack(img, H, W, K, sig, 4.0, pol, st);
        ora_log_direct(img, H, W, K, sig, 4.0, pol, st2);
        double d = 0.0;
        for (size_t i = 0; i < N * (size_t)K; ++i) d = fmax(d, fabs(st[i] - st2[i]));
        check(d < 1e-9, "separable and 2-D stacks agree");
        double p = ora_log_point(img, H, W, sig[K - 1], 4.0, pol, H - 1, W - 1);
        check(fabs(p - st[(size_t)(K - 1) * N + N - 1]) < 1e-9, "log_point matches the stack");
    }
    int32_t *ykx = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(cap > 0 ? cap : 1));
    double *resp = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    long n = ora_candidates(st, K, H, W, -1.0, ykx, resp, cap);
    check(n >= 0, "candidate count");
    long kept = n < cap ? n : cap;
    uint8_t *mask = (uint8_t *)malloc(N * K);
    ora_ambiguous(st, K, H, W, 0.0, 1e-4, mask);
    uint8_t *keep = (uint8_t *)malloc((size_t)(kept > 0 ? kept : 1));
    ora_prune(ykx, sig, kept, 0.5, keep);
    ora_prune(ykx, sig, 0, 0.5, keep);
    double *L = (double *)malloc(sizeof(double) * N * K);
    double *M = (double *)malloc(sizeof(double) * N);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * N);
    ora_gauss_stack(img, H, W, K, sig, 4.0, L);
    long nd = ora_dog_criterion(L, H, W, K, sig, -1e300, M, idx, ykx, cap);
    check(nd >= 0, "DoG count");
    free(img);
    free(st);
    free(st2);
    free(ykx);
    free(resp);
    free(mask);
    free(keep);
    free(L);
    free(M);
    free(idx);
}

int main(void)
{
    ora_set_threads(1);
    check(ora_threads() >= 1, "thread count");
    for (long u = -40; u < 40; ++u) {
        long e = ora_ext(u, 3);
        check(e >= 0 && e < 3, "reflection stays inside");
    }
    check(ora_ext(0, 1) == 0 && ora_ext(-7, 1) == 0, "one-sample reflection");
    for (int i = 0; i < 6; ++i) {
        double s = 0.25 + 2.5 * i;
        int R = ora_radius(s, 4.0);
        check(R >= 0, "radius");
        size_t n = (size_t)(2 * R + 1);  /* two-sided taps, j = -R .. R */
        double *g = (double *)malloc(sizeof(double) * n), *h = (double *)malloc(sizeof(double) * n);
        double *gd = (double *)malloc(sizeof(double) * n), *hd = (double *)malloc(sizeof(double) * n);
        ora_taps(s, R, g, h);
        ora_dtaps(s, R, gd, hd);
        double z = 0.0;
        for (size_t j = 0; j < n; ++j) z += g[j];
        check(fabs(z - 1.0) < 1e-12, "unit-sum Gaussian taps");
        free(g);
        free(h);
        free(gd);
        free(hd);
    }
    /* shapes: one pixel, one row, one column, radii far above the size */
    const double sig_small[3] = {0.5, 1.0, 2.0};
    const double sig_wide[3] = {1.0, 5.0, 9.0};
    detector_case(1, 1, 3, sig_small, 4);
    detector_case(1, 9, 3, sig_wide, 2);
    detector_case(7, 1, 3, sig_wide, 64);
    detector_case(5, 6, 3, sig_wide, 1000);
    detector_case(16, 13, 3, sig_small, 3);
    detector_case(16, 13, 3, sig_small, 0);

    /* constant image: no response */
    {
        double c[35], st[3 * 35];
        for (int i = 0; i < 35; ++i) c[i] = 0.7;
        ora_log_stack(c, 5, 7, 3, sig_wide, 4.0, 0, st);
        double m = 0.0;
        for (int i = 0; i < 3 * 35; ++i) m = fmax(m, fabs(st[i]));
        check(m < 1e-12, "constant image has no response");
    }
    check(fabs(ora_overlap(3, 4, 2, 3, 4, 2) - 1.0) < 1e-12, "self overlap is 1");
    check(ora_overlap(0, 0, 1, 10, 10, 1) == 0.0, "disjoint overlap is 0");
    check(fabs(ora_overlap(0, 0, 1, 0, 0.5, 4) - 1.0) < 1e-12, "contained overlap is 1");

    /* soft score and its gradient, adjoint */
    {
        const int B = 2, H = 9, W = 7, K = 3;
        int radii[3];
        for (int k = 0; k < K; ++k) radii[k] = ora_radius(sig_wide[k], 4.0);
        double *imgs = field(B * H * W, 99u);
        double scores[2], gbar[2] = {1.0, -0.5}, dsig[3];
        double *dimgs = (double *)malloc(sizeof(double) * B * H * W);
        ora_soft_score(imgs, B, H, W, K, sig_wide, radii, 50.0, 0.1, scores);
        ora_soft_score_grad(imgs, B, H, W, K, sig_wide, radii, 50.0, 0.1, gbar, dimgs, dsig);
        check(scores[0] > 0.0 && scores[1] > 0.0, "softplus sums are positive");
        double *adj = (double *)malloc(sizeof(double) * H * W);
        ora_log_adjoint(imgs, H, W, 9.0, 4.0, 1, adj);
        free(adj);
        free(imgs);
        free(dimgs);
    }

    /* stretch on pitched 8-bit rows */
    {
        const int H = 5, W = 6;
        const long pitch = 9;
        uint8_t img[5 * 9];
        uint64_t s = 5u;
        for (int i = 0; i < H * (int)pitch; ++i) img[i] = (uint8_t)(next_u(&s) * 256.0);
        int64_t hist[256];
        int lo, hi;
        ora_stretch_levels(img, H, W, pitch, hist, &lo, &hi);
        int64_t tot = 0;
        for (int v = 0; v < 256; ++v) tot += hist[v];
        check(tot == (int64_t)H * W, "histogram counts every pixel once");
        double out[30];
        ora_stretch(img, H, W, pitch, out, &lo, &hi);
        for (int i = 0; i < H * W; ++i) check(out[i] >= 0.0 && out[i] <= 1.0, "stretched range");
        uint8_t flat[4] = {9, 9, 9, 9};
        ora_stretch(flat, 1, 4, 4, out, &lo, &hi);
        check(out[0] == 0.0 && lo == hi, "flat image maps to 0");
    }
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
