"""Pins of the oracle's histogram stretch (section 3; Algorithm 1, first
step: 0.175% of the pixels saturated at each end, the rest mapped linearly
to [0, 1]), against definitions that do not go through its histogram walk:
order statistics of the sorted pixels, saturation counts, a hand-built
case and the constant image."""
import zlib

import numpy as np
import pytest

import oracle


def sorted_levels(img):
    """low / high as order statistics: with c = ceil(0.00175 N) (in
    integers), low is the c-th smallest pixel and high the c-th largest."""
    s = np.sort(img.ravel())
    n = s.size
    c = (175 * n + 99999) // 100000
    return int(s[c - 1]), int(s[n - c])


@pytest.mark.parametrize("shape,kind", [((37, 53), "uniform"), ((200, 311), "skewed"),
                                        ((1, 1), "uniform"), ((3, 700), "bimodal"),
                                        ((512, 512), "narrow"), ((64, 65), "sparse")])
def test_levels_are_order_statistics(shape, kind):
    rng = np.random.default_rng(zlib.crc32(f"{shape}{kind}".encode()))
    if kind == "uniform":
        img = rng.integers(0, 256, shape)
    elif kind == "skewed":
        img = np.minimum(255, rng.exponential(20.0, shape)).astype(int)
    elif kind == "bimodal":
        img = np.where(rng.random(shape) < 0.5, rng.integers(10, 30, shape),
                       rng.integers(200, 240, shape))
    elif kind == "narrow":
        img = rng.integers(118, 121, shape)
    else:
        img = np.zeros(shape, int)
        img[rng.random(shape) < 0.01] = 255
    img = img.astype(np.uint8)
    lo, hi, hist = oracle.stretch_levels(img)
    assert (lo, hi) == sorted_levels(img)
    assert np.array_equal(hist, np.bincount(img.ravel(), minlength=256))


def test_saturated_fractions():
    """At least 0.175% of the pixels map to 0 and to 1, and the pixels below
    low (above high) are fewer than 0.175%: the saturated sets are the
    smallest ones that reach the fraction."""
    rng = np.random.default_rng(5)
    img = np.clip(rng.normal(120, 30, (300, 400)), 0, 255).astype(np.uint8)
    lo, hi, _ = oracle.stretch_levels(img)
    out = oracle.stretch(img)
    n, q = img.size, 0.00175 * img.size
    assert (out == 0).sum() >= q and (out == 1).sum() >= q
    assert (img < lo).sum() < q and (img > hi).sum() < q
    assert out.min() == 0.0 and out.max() == 1.0
    # monotone in the code, linear between the levels
    mid = (img > lo) & (img < hi)
    assert np.all(np.diff(out.ravel()[np.argsort(img.ravel(), kind="stable")]) >= 0)
    v = img[mid].astype(np.float64)
    assert np.allclose(out[mid] * (hi - lo) + lo, v, rtol=0, atol=1e-12)
    assert n == out.size


def test_hand_built_levels():
    """1000 pixels: q = 1.75, so two pixels are needed at each end."""
    img = np.full(1000, 150, np.uint8)
    img[0], img[1], img[2] = 0, 5, 9          # darkest three
    img[3], img[4] = 250, 240                 # lightest two
    img[5:500] = 100
    lo, hi, _ = oracle.stretch_levels(img.reshape(10, 100))
    assert (lo, hi) == (5, 240)
    out = oracle.stretch(img.reshape(10, 100)).ravel()
    assert out[0] == 0.0 and out[1] == 0.0 and out[2] == pytest.approx(4 / 235)
    assert out[3] == 1.0 and out[4] == 1.0
    assert out[5] == pytest.approx(95 / 235)


def test_constant_image_maps_to_zero():
    img = np.full((40, 30), 77, np.uint8)
    lo, hi, _ = oracle.stretch_levels(img)
    assert lo == hi == 77
    assert not oracle.stretch(img).any()
