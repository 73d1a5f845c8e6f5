"""Matrix-core (split-FP16 MFMA) LoG stack of 8-bit tiles against the FP64
oracle.

The scale list reaches every kernel instantiation (row-pass, column-pass
K-blocks): radius 0 and 4 (1, 1), 9 and 18 (2, 2), 28 and 36 (3, 3), 46 and
54 (4, 4), and 60, above the matrix-core limit of 56, which the strip kernel
computes in the same call.  Shapes cover tiles narrower than
the taps (repeated reflection), widths that are not multiples of 16 or 4,
row pitches that are not multiples of 8 (the per-element load path) and the
aligned fast path.  Tolerance: each plane within 1e-5 of its largest oracle
value, the bound every LoG stack of the library meets."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import synth

from parity import as_set, compare_candidates, plane_rel_err

pytestmark = pytest.mark.gpu

STACK_TOL = 1e-5
SIGMAS = [0.1, 1.0, 2.2, 4.5, 7.0, 9.0, 11.5, 13.5, 15.0]
RADII = [0, 4, 9, 18, 28, 36, 46, 54, 60]


def run_stack(plan, img: np.ndarray, pitch: int | None = None) -> np.ndarray:
    h, w = img.shape
    pitch = w if pitch is None else pitch
    buf = np.zeros((h, pitch), np.uint8)
    buf[:, :w] = img
    t = torch.from_numpy(buf).to(plan.device)[:, :w]
    return plan.detect(t, return_stack=True).stack.cpu().numpy()


def u8_plan(max_hw, sigmas=SIGMAS, **kw):
    from paper_2108_12050_amd import Plan
    args = dict(sigmas=list(sigmas), threshold=0.05, overlap=1.0, dtype="u8",
                max_h=max_hw, max_w=max_hw)
    args.update(kw)
    return Plan(**args)


def test_radii_reach_every_instantiation():
    assert [oracle.radius(float(np.float32(s))) for s in SIGMAS] == RADII


@pytest.mark.parametrize("h,w,pitch", [(37, 23, 23), (129, 200, 200), (130, 261, 261),
                                       (260, 512, 520), (1, 50, 50), (50, 1, 1),
                                       (96, 300, 300)])
def test_u8_stack_matches_oracle(h, w, pitch):
    print(f"u8 stack {h}x{w} pitch {pitch}", flush=True)
    img = synth.sem_tile(h * 7 + w, psf_sigma=1.0, H=h, W=w)
    plan = u8_plan(512)
    st = run_stack(plan, img, pitch)
    I = oracle.to_f64(img)
    ora = oracle.log_stack(I, np.float64(np.float32(SIGMAS)))
    if min(h, w) > 1:
        err = plane_rel_err(st, ora)
        assert err.max() <= STACK_TOL, err
    else:
        # One row (or column): every window along the other axis reflects the
        # same line, the second-derivative taps cancel against it, and the
        # response is small next to the intermediates; the bound is taken
        # against the image scale, as for the other degenerate shapes.
        err = np.abs(st - ora).reshape(len(ora), -1).max(1)
        assert err.max() <= STACK_TOL * max(np.abs(ora).max(), np.abs(I).max()), err


def test_u8_extreme_codes():
    """Codes 0 and 255 only (the largest intermediates the tap scaling allows
    for), on a checkerboard of 5-pixel cells and a single bright pixel."""
    plan = u8_plan(128)
    yy, xx = np.mgrid[0:100, 0:90]
    board = np.where(((yy // 5) + (xx // 5)) % 2 == 0, 255, 0).astype(np.uint8)
    dot = np.zeros((64, 64), np.uint8)
    dot[31, 40] = 255
    for img in (board, dot):
        st = run_stack(plan, img)
        ora = oracle.log_stack(oracle.to_f64(img), np.float64(np.float32(SIGMAS)))
        assert plane_rel_err(st, ora).max() <= STACK_TOL


def test_u8_candidates_and_dark_polarity():
    sig = oracle.linear_sigmas(10, 1.0, 10.0)
    img = synth.sem_tile(3, psf_sigma=2.0, H=384, W=320)
    tau = float(np.float32(0.05))
    for pol, s in (("bright", 0), ("dark", 1)):
        from paper_2108_12050_amd import Plan
        plan = Plan(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, overlap=1.0,
                    dtype="u8", polarity=pol, max_h=512, max_w=512)
        t = torch.from_numpy(img).to(plan.device)
        d = plan.detect(t, return_stack=True)
        st = d.stack.cpu().numpy()
        ora = oracle.log_stack(oracle.to_f64(img), sig, polarity=s)
        assert plane_rel_err(st, ora).max() <= STACK_TOL
        ykx, _ = oracle.candidates(ora, tau)
        compare_candidates(st, as_set(d.yxk.cpu().numpy()), ora, as_set(ykx), tau)
        assert len(ykx) > 20


def test_segments_and_tall_tiles():
    """Tall tiles split into several row segments per wave: segment seams must
    not show.  Height 1100 is not a multiple of 16."""
    sig = oracle.linear_sigmas(10, 1.0, 10.0)
    img = synth.sem_tile(8, psf_sigma=0.0, H=1100, W=96)
    plan = u8_plan(1100, sigmas=sig)
    st = run_stack(plan, img)
    ora = oracle.log_stack(oracle.to_f64(img), sig)
    assert plane_rel_err(st, ora).max() <= STACK_TOL
