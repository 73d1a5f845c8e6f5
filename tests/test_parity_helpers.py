"""CPU pins of the whole-tile helpers the full-size GPU tests use: the
strip-wise prune equals the oracle's prune of the whole list, and the
candidate rule applied to a stack's own values equals the oracle's
candidate search (ties included)."""
import numpy as np

import oracle
from paper_2108_12050_amd import synth

from parity import own_maxima, strip_prune

SIG10 = oracle.linear_sigmas(10, 1.0, 10.0)


def _stack_and_candidates(img, tau):
    st = oracle.log_stack(oracle.to_f64(img), SIG10)
    c, _ = oracle.candidates(st, tau)
    return st, c.astype(np.int64)


def test_strip_prune_equals_whole_list_prune():
    tau = float(np.float32(0.05))
    img = synth.sem_tile(0, psf_sigma=1.0, H=320, W=288)
    _, cand = _stack_and_candidates(img, tau)
    whole = cand[oracle.prune(cand, SIG10, 0.5)]
    assert 0 < len(whole) < len(cand)
    for step in (16, 64, 128):
        np.testing.assert_array_equal(strip_prune(cand, SIG10, 0.5, 320, step=step), whole)


def test_strip_prune_needs_its_margin():
    """A margin below the overlap reach drops dominators at strip seams: the
    check is sensitive to the margin it relies on."""
    tau = float(np.float32(0.05))
    img = synth.sem_tile(0, psf_sigma=1.0, H=320, W=288)
    _, cand = _stack_and_candidates(img, tau)
    whole = cand[oracle.prune(cand, SIG10, 0.5)]
    thin = strip_prune(cand, SIG10, 0.5, 320, step=16, margin=0)
    assert len(thin) > len(whole)


def test_own_maxima_equals_oracle_candidates():
    for img, tau in ((synth.plain_tile(1, H=200, W=232), 0.1),
                     (synth.sem_tile(2, psf_sigma=0.0, H=160, W=176), 0.05)):
        tau = float(np.float32(tau))
        st, cand = _stack_and_candidates(img, tau)
        np.testing.assert_array_equal(own_maxima(st, tau), cand)


def test_own_maxima_keeps_plateaus_and_borders():
    """Equal neighbours both pass the equality test; border voxels see -inf
    outside the volume; the threshold is strict."""
    st = np.zeros((3, 5, 6), np.float32)
    st[1, 2, 2] = st[1, 2, 3] = 1.0      # plateau of two
    st[0, 0, 0] = 0.5                     # corner voxel
    st[2, 4, 5] = 0.25                    # exactly at the threshold: rejected
    got = own_maxima(st, 0.25)
    np.testing.assert_array_equal(got, [[0, 0, 0], [2, 2, 1], [2, 3, 1]])
