"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (Gaussian kernel of section 2.2, the scale-normalised response of a
Gaussian blob, Laplacians of polynomials), invariances (translation, flips,
self-adjointness under half-sample reflection), library routines for special
cases (numpy/scipy reflect-mode correlation, scipy maximum filter as the
maxpool-equality test of section 3), textbook geometry (circle-circle lens
area) and brute force on tiny inputs.
"""
import math

import numpy as np
import pytest

SIG10 = np.arange(1.0, 11.0)


# ---------------------------------------------------------------- taps / ext

@pytest.mark.parametrize("sigma", [0.6, 1.0, 2.5, 4.0, 7.3, 10.0])
def test_taps_shape_and_moments(ora, sigma):
    R = ora.radius(sigma, 4.0)
    assert R == math.floor(4.0 * sigma + 0.5)
    g, h = ora.taps(sigma, R)
    j = np.arange(-R, R + 1)
    # Gaussian of section 2.2: g_j / g_0 = exp(-j^2 / (2 sigma^2))
    np.testing.assert_allclose(g / g[R], np.exp(-j ** 2 / (2 * sigma ** 2)), rtol=1e-14)
    assert abs(g.sum() - 1.0) < 1e-15
    assert abs(h.sum()) < 1e-15 * np.abs(h).sum() * 10
    np.testing.assert_array_equal(g, g[::-1])
    np.testing.assert_array_equal(h, h[::-1])
    # Heat-equation identity of the scale derivative: d g_j / d sigma equals
    # sigma * h_j (h = 2 dg/d(sigma^2)), checked by central differences in
    # sigma at fixed support.
    d = 1e-5
    gp, _ = ora.taps(sigma + d, R)
    gm, _ = ora.taps(sigma - d, R)
    np.testing.assert_allclose((gp - gm) / (2 * d), sigma * h, rtol=0, atol=1e-8)
    # Second moment of the second-derivative taps -> 2 (d^2/dx^2 of x^2) as
    # sampling and truncation errors vanish; 4-sigma truncation keeps it
    # within 2 percent for sigma >= 1.
    if sigma >= 1.0:
        assert abs((j ** 2 * h).sum() - 2.0) < 2e-2


@pytest.mark.parametrize("n", [1, 2, 3, 7])
def test_ext_is_half_sample_symmetric(ora, n):
    pad = 3 * n + 5
    ref = np.pad(np.arange(n), (pad, pad), mode="symmetric")
    got = [ora.ext(u, n) for u in range(-pad, n + pad)]
    np.testing.assert_array_equal(got, ref)


# ---------------------------------------------------------------- LoG stack

@pytest.mark.parametrize("shape", [(1, 1), (3, 2), (20, 17), (64, 48)])
def test_constant_image_has_zero_response(ora, shape):
    c = 0.37
    st = ora.log_stack(np.full(shape, c), SIG10)
    assert np.abs(st).max() <= 1e-14 * c


@pytest.mark.parametrize("t", [1.5, 2.5, 4.0, 6.0, 8.0])
def test_isolated_blob_matches_closed_form(ora, t):
    """-sigma^2 Lap (G_sigma * A exp(-r^2/2t^2)) = A sigma^2 t^2 (2 - r^2/s^2)
    exp(-r^2/2s^2) / s^4 with s^2 = sigma^2 + t^2 (Gaussians compose by adding
    variances; section 2.2's scale space)."""
    H = W = 161
    c = 80
    A = 0.7
    y, x = np.mgrid[0:H, 0:W]
    img = A * np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * t * t))
    st = ora.log_stack(img, SIG10)
    for k, s in enumerate(SIG10):
        s2 = s * s + t * t
        for (dy, dx) in [(0, 0), (0, 3), (2, 2), (5, 1)]:
            r2 = dy * dy + dx * dx
            cf = A * s * s * t * t * (2 - r2 / s2) * math.exp(-r2 / (2 * s2)) / s2 ** 2
            got = st[k, c + dy, c + dx]
            # sampling + 4-sigma truncation error of the discrete operator
            assert abs(got - cf) <= 5e-3 * A / 2, (t, s, dy, dx, got, cf)
        centre = 2 * A * s * s * t * t / s2 ** 2
        assert abs(st[k, c, c] / centre - 1) < 5e-3


@pytest.mark.parametrize("t", [2.0, 3.0, 5.0, 7.0, 9.0])
def test_scale_selection_peaks_at_blob_scale(ora, t):
    """A feature of scale t responds most strongly at sigma = t (section 2.2);
    the closed-form centre value 2 A sigma^2 t^2/(sigma^2+t^2)^2 peaks at
    sigma = t with value A/2."""
    H = W = 201
    c = 100
    y, x = np.mgrid[0:H, 0:W]
    img = np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * t * t))
    st = ora.log_stack(img, SIG10)
    centre = st[:, c, c]
    assert SIG10[int(np.argmax(centre))] == t
    assert abs(centre.max() - 0.5) < 5e-3


@pytest.mark.parametrize("shape,sig", [((7, 5), [1.0, 3.0]), ((12, 9), [0.8, 2.0, 2.6]),
                                       ((3, 40), [1.0, 5.0]), ((1, 6), [2.0])])
def test_separable_equals_direct_2d(ora, shape, sig):
    rng = np.random.default_rng(1)
    img = rng.uniform(-1, 1, shape)
    a = ora.log_stack(img, sig)
    b = ora.log_direct(img, sig)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("shape,sig", [((9, 13), [1.0, 2.0, 4.0]), ((40, 33), [1.0, 3.5, 10.0])])
def test_matches_scipy_reflect_correlation(ora, shape, sig):
    """scipy.ndimage's 'reflect' mode is the half-sample extension; with the
    Gaussian taps built here from their definition the separable LoG must
    agree with the oracle, also when the kernel is longer than the image."""
    from scipy.ndimage import correlate1d
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 1, shape)
    st = ora.log_stack(img, sig)
    for k, s in enumerate(sig):
        R = int(math.floor(4 * s + 0.5))
        j = np.arange(-R, R + 1)
        e = np.exp(-j ** 2 / (2 * s * s))
        g = e / e.sum()
        V = (j ** 2 * g).sum()
        h = (j ** 2 - V) * g / s ** 4
        A = correlate1d(img, g, axis=1, mode="reflect")
        B = correlate1d(img, h, axis=1, mode="reflect")
        lap = correlate1d(A, h, axis=0, mode="reflect") + correlate1d(B, g, axis=0, mode="reflect")
        np.testing.assert_allclose(st[k], -s * s * lap, rtol=0, atol=1e-13)


def test_polynomial_images(ora):
    """On the interior the scale-normalised Laplacian of x^2 is 2 sigma^2, of
    x^2 + y^2 is 4 sigma^2, and of x*y and linear ramps is 0 (up to the 4-sigma
    truncation of the kernel moments)."""
    H, W = 101, 97
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    y -= 50.0
    x -= 48.0
    sig = [1.0, 2.0, 3.0]
    cases = [(x ** 2, 2.0), (x ** 2 + y ** 2, 4.0), (x * y, 0.0), (3 * x - 2 * y + 1, 0.0)]
    for img, lap in cases:
        st = ora.log_stack(img, sig, polarity=1)
        for k, s in enumerate(sig):
            R = int(math.floor(4 * s + 0.5))
            inner = st[k, R:H - R, R:W - R]
            # kernel moments carry the 4-sigma truncation deficit (< 2 percent)
            np.testing.assert_allclose(inner, lap * s * s, rtol=0, atol=2e-2 * max(1, lap) * s * s)


def test_translation_equivariance(ora):
    rng = np.random.default_rng(3)
    big = rng.uniform(0, 1, (90, 80))
    sig = [1.0, 2.0, 4.0]
    dy, dx = 5, 7
    a = ora.log_stack(big[:70, :60], sig)
    b = ora.log_stack(big[dy:dy + 70, dx:dx + 60], sig)
    R = 16
    np.testing.assert_allclose(a[:, R + dy:70 - R, R + dx:60 - R],
                               b[:, R:70 - R - dy, R:60 - R - dx], rtol=0, atol=1e-13)


def test_flip_and_transpose_equivariance(ora):
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 1, (31, 23))
    sig = [1.0, 3.0, 9.0]
    a = ora.log_stack(img, sig)
    np.testing.assert_allclose(ora.log_stack(img[:, ::-1], sig), a[:, :, ::-1], atol=1e-13)
    np.testing.assert_allclose(ora.log_stack(img[::-1, :], sig), a[:, ::-1, :], atol=1e-13)
    np.testing.assert_allclose(ora.log_stack(img.T.copy(), sig), a.transpose(0, 2, 1), atol=1e-13)


@pytest.mark.parametrize("shape,sigma", [((5, 4), 1.0), ((13, 9), 3.0), ((20, 31), 10.0)])
def test_operator_is_self_adjoint(ora, shape, sigma):
    """Under the half-sample extension each 1-D border-handled convolution
    with a symmetric kernel is a symmetric matrix, so the LoG operator equals
    its adjoint, which the oracle forms by explicit scatter."""
    rng = np.random.default_rng(5)
    u = rng.normal(size=shape)
    v = rng.normal(size=shape)
    Cu = ora.log_stack(u, [sigma])[0]
    CTv = ora.log_adjoint(v, sigma)
    lhs = (Cu * v).sum()
    rhs = (u * CTv).sum()
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    np.testing.assert_allclose(CTv, ora.log_stack(v, [sigma])[0], rtol=0, atol=1e-12)


def test_scale_partition_invariance(ora):
    """Computing the scales in separate groups (the multi-device partition of
    section 5) leaves every plane unchanged."""
    rng = np.random.default_rng(6)
    img = rng.uniform(0, 1, (40, 36))
    full = ora.log_stack(img, SIG10)
    parts = np.concatenate([ora.log_stack(img, SIG10[:3]), ora.log_stack(img, SIG10[3:7]),
                            ora.log_stack(img, SIG10[7:])])
    np.testing.assert_array_equal(full, parts)


def test_point_evaluation_matches_stack(ora):
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 1, (37, 29))
    st = ora.log_stack(img, [1.0, 2.5])
    for (y, x) in [(0, 0), (36, 28), (18, 3), (5, 20)]:
        for k, s in enumerate([1.0, 2.5]):
            assert abs(ora.log_point(img, s, y, x) - st[k, y, x]) < 1e-13


def test_u8_input_is_scaled(ora):
    u = np.arange(0, 256, dtype=np.uint8).reshape(16, 16)
    np.testing.assert_array_equal(ora.to_f64(u), u.astype(np.float64) / 255.0)


def test_linear_scale_grid(ora):
    """t_i = min_t + (i-1) delta_t, delta_t = (max_t - min_t)/n, K = n+1."""
    np.testing.assert_array_equal(ora.linear_sigmas(10, 1.0, 10.0), SIG10)
    g = ora.linear_sigmas(5, 1.5, 3.5)
    np.testing.assert_allclose(g, [1.5, 2.0, 2.5, 3.0, 3.5])
    assert ora.linear_sigmas(1, 2.0, 9.0).tolist() == [2.0]


# ---------------------------------------------------------------- maxima

def _maxpool_candidates(st, tau):
    """Maxpool-equality maxima (section 3) with scipy's maximum filter over a
    3x3x3 window, borders padded with -inf, then the strict threshold."""
    from scipy.ndimage import maximum_filter
    m = maximum_filter(st, size=3, mode="constant", cval=-np.inf)
    k, y, x = np.nonzero((st >= m) & (st > tau))
    order = np.lexsort((k, x, y))
    return np.stack([y[order], x[order], k[order]], 1)


@pytest.mark.parametrize("seed", range(6))
def test_candidates_match_maxpool_equality(ora, seed):
    rng = np.random.default_rng(seed)
    shape = [(3, 6, 7), (1, 5, 5), (4, 1, 9), (2, 8, 3), (5, 4, 4), (3, 10, 12)][seed]
    # small integers force plateaus and ties
    st = rng.integers(0, 4, shape).astype(np.float64)
    tau = 1.5
    ykx, resp = ora.candidates(st, tau)
    ref = _maxpool_candidates(st, tau)
    np.testing.assert_array_equal(ykx, ref.reshape(-1, 3))
    np.testing.assert_array_equal(resp, st[ykx[:, 2], ykx[:, 0], ykx[:, 1]])


def test_single_blob_gives_one_record_at_its_centre(ora):
    H = W = 129
    y, x = np.mgrid[0:H, 0:W]
    img = 0.1 + 0.8 * np.exp(-((y - 64) ** 2 + (x - 60) ** 2) / (2 * 4.0 ** 2))
    d = ora.detect(img, SIG10, tau=0.1, theta=0.5)
    assert d["count"] == 1
    assert d["blobs"].tolist() == [[64, 60, 3]]
    assert abs(d["blob_resp"][0] - 0.4) < 2e-3


def test_ambiguity_margin(ora):
    st = np.zeros((1, 3, 3))
    st[0, 1, 1] = 0.5
    st[0, 1, 2] = 0.5 - 5e-5      # near-tie with the maximum
    st[0, 0, 0] = 0.10003         # near tau but below its neighbour... not a max
    n, m = ora.ambiguous(st, 0.1, 1e-4, mask=True)
    assert m[0, 1, 1] and m[0, 1, 2]
    assert not m[0, 0, 0] and n == 2
    st[0, 1, 2] = 0.3
    assert ora.ambiguous(st, 0.1, 1e-4) == 0
    st2 = np.zeros((1, 1, 1)) + 0.10005   # lone voxel just above tau
    assert ora.ambiguous(st2, 0.1, 1e-4) == 1


# ---------------------------------------------------------------- prune

@pytest.mark.parametrize("q", [0.0, 0.1, 0.37, 0.5, 0.8, 0.99])
def test_overlap_equal_radii_closed_form(ora, q):
    r = 3.0
    d = 2 * r * q
    ref = (2 / math.pi) * (math.acos(q) - q * math.sqrt(1 - q * q))
    assert abs(ora.overlap(0, 0, r, 0, d, r) - ref) < 1e-12


def test_overlap_limits(ora):
    assert ora.overlap(0, 0, 2, 0, 5, 3) == 0.0        # touching
    assert ora.overlap(0, 0, 2, 0, 6, 3) == 0.0
    assert ora.overlap(0, 0, 2, 0, 1, 3) == 1.0        # inside
    assert ora.overlap(4, 4, 5, 4, 4, 1) == 1.0        # concentric


@pytest.mark.parametrize("ra,rb,d", [(2.0, 3.0, 2.5), (1.4, 9.0, 8.0), (5.0, 5.5, 1.2)])
def test_overlap_unequal_radii_by_integration(ora, ra, rb, d):
    n = 4000
    lo, hi = -ra, ra
    s = (np.arange(n) + 0.5) / n * (hi - lo) + lo
    Y, X = np.meshgrid(s, s, indexing="ij")
    ina = X ** 2 + Y ** 2 <= ra * ra
    inb = (X - d) ** 2 + Y ** 2 <= rb * rb
    area = (ina & inb).sum() * ((hi - lo) / n) ** 2
    ref = area / (math.pi * min(ra, rb) ** 2)
    assert abs(ora.overlap(0, 0, ra, 0, d, rb) - ref) < 2e-3


def test_prune_rule_hand_cases(ora):
    sig = SIG10
    r = math.sqrt(2) * 4.0   # scale index 3
    # same scale: overlap > 0.5 iff d < d*, with d* the equal-radii crossing
    dstar = 2 * r * 0.4040   # (2/pi)(acos q - q sqrt(1-q^2)) = 0.5 at q ~ 0.40397
    close = int(math.floor(dstar - 0.2))
    far = int(math.ceil(dstar + 0.2))
    keep = ora.prune([[10, 10, 3], [10, 10 + close, 3]], sig, 0.5)
    assert keep.tolist() == [True, False]         # smaller (y, x) wins a tie of scale
    keep = ora.prune([[10, 10, 3], [10, 10 + far, 3]], sig, 0.5)
    assert keep.tolist() == [True, True]
    # larger scale removes a smaller one inside it, whatever the order
    keep = ora.prune([[5, 5, 0], [6, 6, 9]], sig, 0.5)
    assert keep.tolist() == [False, True]
    # one-shot: a removed blob still removes the ones it dominates
    keep = ora.prune([[20, 20, 9], [20, 22, 5], [20, 24, 2]], sig, 0.5)
    assert keep.tolist() == [True, False, False]
    # theta >= 1 never removes
    assert ora.prune([[5, 5, 0], [5, 5, 9]], sig, 1.0).tolist() == [True, True]


def test_prune_against_brute_force_geometry(ora):
    """Random lists: the prune decision equals the rule evaluated with an
    overlap computed by grid integration (away from the 0.5 boundary)."""
    rng = np.random.default_rng(11)
    n = 40
    ykx = np.stack([rng.integers(0, 40, n), rng.integers(0, 40, n), rng.integers(0, 4, n)], 1)
    ykx = np.unique(ykx, axis=0)
    sig = np.array([1.0, 2.0, 3.0, 4.0])
    keep = ora.prune(ykx, sig, 0.5)

    def ov_grid(a, b):
        ya, xa, ka = a
        yb, xb, kb = b
        ra, rb = math.sqrt(2) * sig[ka], math.sqrt(2) * sig[kb]
        rs = min(ra, rb)
        cy, cx = (ya, xa) if ra <= rb else (yb, xb)
        oy, ox, ro = (yb, xb, rb) if ra <= rb else (ya, xa, ra)
        m = 600
        s = (np.arange(m) + 0.5) / m * 2 * rs - rs
        Y, X = np.meshgrid(s + cy, s + cx, indexing="ij")
        ins = (Y - cy) ** 2 + (X - cx) ** 2 <= rs * rs
        ino = (Y - oy) ** 2 + (X - ox) ** 2 <= ro * ro
        return (ins & ino).sum() * (2 * rs / m) ** 2 / (math.pi * rs * rs)

    decided = 0
    for bi, b in enumerate(ykx):
        removed, unsure = False, False
        for ai, a in enumerate(ykx):
            if ai == bi:
                continue
            dom = a[2] > b[2] or (a[2] == b[2] and (a[0], a[1]) < (b[0], b[1]))
            if not dom:
                continue
            o = ov_grid(a, b)
            if abs(o - 0.5) < 0.02:
                unsure = True       # grid integration cannot call this pair
            elif o > 0.5:
                removed = True
        if removed or not unsure:
            assert keep[bi] == (not removed)
            decided += 1
    assert decided >= len(ykx) - 3 and (~keep).sum() >= 3


# ---------------------------------------------------------------- soft score

def test_soft_score_constant_image(ora):
    beta, tau = 50.0, 0.05
    img = np.full((2, 17, 23), 0.4)
    S = ora.soft_score(img, SIG10[:4], beta, tau)
    np.testing.assert_allclose(S, math.log1p(math.exp(-beta * tau)), rtol=1e-14)
    dI, ds = ora.soft_score_grad(img, SIG10[:4], beta, tau)
    assert np.abs(dI).max() < 1e-15 and np.abs(ds).max() < 1e-15


def test_soft_score_is_mean_softplus_of_stack(ora):
    rng = np.random.default_rng(8)
    img = rng.uniform(0, 1, (2, 21, 19))
    sig = [1.0, 2.0, 3.5]
    beta, tau = 50.0, 0.05
    S = ora.soft_score(img, sig, beta, tau)
    for b in range(2):
        r = np.abs(ora.log_stack(img[b], sig))
        z = beta * (r - tau)
        ref = np.mean(np.logaddexp(0.0, z))
        assert abs(S[b] - ref) < 1e-13


def _kink_crossed(ora, imgs, sig_p, sig_m):
    """True if some response r changes sign between the two perturbed inputs
    (|r| has a kink at 0, where central differences are only O(h))."""
    for b in range(imgs[0].shape[0]):
        a = ora.log_stack(imgs[0][b], sig_p)
        c = ora.log_stack(imgs[1][b], sig_m)
        if np.any(np.sign(a) != np.sign(c)):
            return True
    return False


def test_soft_score_gradient_by_central_differences(ora):
    """Central differences in FP64: every sigma and 8 random image directions
    within 1e-4 relative of the analytic gradient (radius held fixed, as the
    derivative is taken with the support frozen).  The step h = 1e-3 is
    checked wherever no response crosses the kink of |r| at 0 within +-h; a
    step of 1e-6 is checked for every component that is kink-free at that
    step (at least the sigmas and 6 of the 8 directions).  FP64 round-off at
    h = 1e-6 is about 1e-10 relative here."""
    rng = np.random.default_rng(9)
    from paper_2108_12050_amd import synth
    imgs = np.stack([synth.blob_field(40 + b, 40, 36, n_blobs=4) for b in range(2)]).astype(np.float64)
    sig = np.array([1.0, 2.0, 3.0, 4.5])
    radii = [ora.radius(s, 4.0) for s in sig]
    beta, tau = 50.0, 0.05
    gbar = np.array([1.0, -0.7])
    dI, ds = ora.soft_score_grad(imgs, sig, beta, tau, gbar, radii=radii)

    def f(I, s):
        return float(np.dot(gbar, ora.soft_score(I, s, beta, tau, radii=radii)))

    checked = {1e-3: 0, 1e-6: 0}
    for h in (1e-3, 1e-6):
        for k in range(len(sig)):
            sp, sm = sig.copy(), sig.copy()
            sp[k] += h
            sm[k] -= h
            if _kink_crossed(ora, (imgs, imgs), sp, sm):
                continue
            checked[h] += 1
            fd = (f(imgs, sp) - f(imgs, sm)) / (2 * h)
            assert abs(fd - ds[k]) <= 1e-4 * abs(ds[k]), (h, k, fd, ds[k])
        for _ in range(8):
            v = rng.normal(size=imgs.shape)
            if _kink_crossed(ora, (imgs + h * v, imgs - h * v), sig, sig):
                continue
            checked[h] += 1
            fd = (f(imgs + h * v, sig) - f(imgs - h * v, sig)) / (2 * h)
            an = float((dI * v).sum())
            assert abs(fd - an) <= 1e-4 * abs(an), (h, fd, an)
    assert checked[1e-3] >= 1 and checked[1e-6] >= 4 + 6, checked


def test_soft_score_gradient_pixelwise_fd(ora):
    """Single-pixel central differences for a few pixels, border included."""
    from paper_2108_12050_amd import synth
    img = synth.blob_field(77, 24, 20, n_blobs=3).astype(np.float64)[None]
    sig = np.array([1.0, 2.0])
    beta, tau = 50.0, 0.05
    dI, _ = ora.soft_score_grad(img, sig, beta, tau)
    h = 1e-3
    for (y, x) in [(0, 0), (23, 19), (11, 7), (3, 18)]:
        p, m = img.copy(), img.copy()
        p[0, y, x] += h
        m[0, y, x] -= h
        fd = (ora.soft_score(p, sig, beta, tau)[0] - ora.soft_score(m, sig, beta, tau)[0]) / (2 * h)
        assert abs(fd - dI[0, y, x]) <= 1e-4 * abs(dI[0, y, x]) + 1e-12, (y, x, fd, dI[0, y, x])


# ---------------------------------------------------------------- workload sanity

def test_defocus_reduces_feature_count(ora):
    """Synthetic analogue of the paper's hypothesis (section 3): on the same
    scene, blurring with a wider PSF leaves fewer blob features."""
    from paper_2108_12050_amd import synth
    counts = []
    for p in [0.0, 1.0, 2.0, 4.0]:
        img = synth.sem_tile(3, psf_sigma=p, H=256, W=256)
        counts.append(ora.detect(img, SIG10, tau=0.05, theta=0.5)["count"])
    assert counts[0] > counts[1] > counts[2] > counts[3], counts
