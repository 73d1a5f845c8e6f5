"""Pins of the oracle's Gaussian planes and of the paper's own criterion
(section 3: DoG of equation "dog", argmax over scale and 3x3 maxpool
equality of equation "argmax", the count of Algorithm 1), against
independent libraries and closed forms."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


@pytest.mark.parametrize("sigma", [0.7, 1.0, 2.5, 6.0, 10.0])
def test_gauss_planes_equal_scipy_gaussian_filter(sigma):
    """scipy's gaussian_filter samples the same Gaussian, truncated at
    int(4 sigma + 0.5), normalised, with half-sample reflection ('reflect')."""
    img = np.random.default_rng(1).random((37, 61))
    L = oracle.gauss_stack(img, [sigma])[0]
    ref = ndimage.gaussian_filter(img, sigma, truncate=4.0, mode="reflect")
    assert np.abs(L - ref).max() < 1e-13


@pytest.mark.parametrize("s,t", [(2.0, 1.0), (3.0, 3.0), (4.0, 7.0)])
def test_isolated_blob_centre_closed_form(s, t):
    """A Gaussian blob A exp(-r^2 / 2 s^2) blurred by G_t has centre value
    A s^2 / (s^2 + t^2) (variances add); the sampled, truncated kernels
    agree to within their discretisation error."""
    n = 129
    yy, xx = np.mgrid[0:n, 0:n] - n // 2
    A = 0.8
    img = A * np.exp(-(yy ** 2 + xx ** 2) / (2 * s * s))
    L = oracle.gauss_stack(img, [t])[0]
    exact = A * s * s / (s * s + t * t)
    assert abs(L[n // 2, n // 2] - exact) < 2e-3 * A


def test_criterion_against_numpy_argmax_and_scipy_maxpool():
    rng = np.random.default_rng(2)
    img = ndimage.gaussian_filter(rng.random((48, 70)), 1.5)
    sig = oracle.linear_sigmas(6, 1.0, 4.0)
    L = oracle.gauss_stack(img, sig)
    tau = -0.01
    d = oracle.dog_criterion(L, sig, tau)
    dog = sig[:-1, None, None] * (L[1:] - L[:-1])
    assert np.array_equal(d["idx"], np.argmax(dog, axis=0))       # first maximum on ties
    assert np.array_equal(d["M"], dog.max(axis=0))
    mp = ndimage.maximum_filter(d["M"], size=3, mode="constant", cval=-np.inf)
    want = np.argwhere((d["M"] >= mp) & (d["M"] > tau))
    assert np.array_equal(d["yxk"][:, :2], want)
    assert np.array_equal(d["yxk"][:, 2], d["idx"][want[:, 0], want[:, 1]])
    assert d["count"] == len(want) > 0


def test_constant_image_counts_every_pixel():
    """Every DoG is 0 (to rounding: every pixel sums the same taps times the
    same value in the same order), so M is a plateau and the maxpool
    equality holds at every pixel (no threshold)."""
    L = oracle.gauss_stack(np.full((20, 30), 0.4), [1.0, 2.0, 3.0])
    d = oracle.dog_criterion(L, [1.0, 2.0, 3.0])
    assert d["count"] == 600 and np.abs(d["M"]).max() < 1e-15
    assert np.unique(d["M"]).size == 1


def test_dark_blob_is_found_at_its_scale():
    """The paper's DoG is positive at dark blobs; for a dark blob of std s the
    scale-normalised response peaks at t = s (section 2.2), so the argmax
    over the forward differences lands within one step of s."""
    n, s = 121, 4.0
    yy, xx = np.mgrid[0:n, 0:n] - n // 2
    img = 0.6 - 0.5 * np.exp(-(yy ** 2 + xx ** 2) / (2 * s * s))
    sig = oracle.linear_sigmas(10, 1.0, 10.0)
    d = oracle.dog_criterion(oracle.gauss_stack(img, sig), sig, tau=1e-3)
    c = n // 2
    hits = [tuple(r) for r in d["yxk"].tolist() if r[0] == c and r[1] == c]
    assert len(hits) == 1
    assert abs(sig[hits[0][2]] - s) <= 1.0
