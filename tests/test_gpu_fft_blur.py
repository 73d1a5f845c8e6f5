"""Frequency-domain scale space (plan mode blur="fft") against the FP64
oracle.

With half-sample symmetric borders the separable sampled-Gaussian and
second-derivative filters of section 2.2 are diagonal in the 2-D DCT-II
basis, so the stack comes out of one forward transform and one weighted
inverse transform per scale, exact for any radius (repeated reflection
included).  The tests compare whole stacks with the oracle's direct
convolution on power-of-two tiles of both input types, radii far above the
tile size, the one-row and one-column tiles, candidate decisions and the
prune, sampled voxels of a 4096 x 4096 tile against the 2-D definition, and
the refusals (sides that are not powers of two, the forms the mode does not
serve).

Tolerance: each plane within 1e-5 of its largest oracle value, the bound
of the direct path.  The transforms run in FP32 with twiddles rounded from
double; a radix-2 pass adds about one rounding of the running spectrum, so
the error grows with log2 of the side (measured: 3.0e-7 to 3.3e-7 of the
plane maximum from 256^2 to 1024^2, f32 and 8-bit).  One-row and one-column
tiles are held to the image scale instead (their responses cancel to
rounding level, as in the direct path's tests)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import _lib, synth

from parity import as_set, compare_candidates, gpu_detect, plane_rel_err

pytestmark = pytest.mark.gpu

FFT_TOL = 1e-5
SIG10 = oracle.linear_sigmas(10, 1.0, 10.0)
TAU = float(np.float32(0.1))
# radii 2, 12, 48, 120, 256: the last three exceed a 64-pixel side
WIDE = [0.5, 3.0, 12.0, 30.0, 64.0]


def fft_plan(max_hw=512, **kw):
    from paper_2108_12050_amd import Plan
    args = dict(sigmas=list(SIG10), threshold=TAU, overlap=0.5, max_h=max_hw, max_w=max_hw,
                blur="fft")
    args.update(kw)
    return Plan(**args)


def stack_of(plan, img: np.ndarray) -> np.ndarray:
    t = torch.from_numpy(np.ascontiguousarray(img)).to(plan.device)
    return plan.detect(t, return_stack=True).stack.cpu().numpy()


def check_stack(st, ora, img):
    if min(img.shape) > 1:
        err = plane_rel_err(st, ora)
        assert err.max() <= FFT_TOL, err
    else:
        err = np.abs(st - ora).reshape(len(ora), -1).max(1)
        assert err.max() <= FFT_TOL * max(np.abs(ora).max(), np.abs(oracle.to_f64(img)).max()), err


@pytest.mark.parametrize("shape", [(64, 64), (128, 256), (256, 128), (512, 512), (2, 2),
                                   (1, 64), (64, 1), (1, 1)])
def test_f32_stack_matches_oracle(shape):
    print(f"fft f32 stack {shape}", flush=True)
    img = synth.blob_field(11 + shape[0] + 3 * shape[1], *shape,
                           n_blobs=max(1, shape[0] * shape[1] // 600))
    plan = fft_plan()
    check_stack(stack_of(plan, img), oracle.log_stack(img, SIG10), img)


@pytest.mark.parametrize("shape", [(64, 64), (256, 512), (1, 128), (128, 1)])
def test_u8_wide_radii_match_oracle(shape):
    """8-bit input, radii up to four times the tile side."""
    print(f"fft u8 wide radii {shape}", flush=True)
    img = synth.sem_tile(7 * shape[0] + shape[1], psf_sigma=1.0, H=shape[0], W=shape[1])
    sig = np.float64(np.float32(WIDE))
    plan = fft_plan(sigmas=WIDE, dtype="u8", threshold=0.05)
    assert plan.radii == [2, 12, 48, 120, 256]
    check_stack(stack_of(plan, img), oracle.log_stack(oracle.to_f64(img), sig), img)


@pytest.mark.parametrize("polarity", ["bright", "dark"])
def test_detection_matches_oracle(polarity):
    """Candidate decisions against the oracle's stack (exact away from
    ambiguous voxels), and the prune exactly over the GPU's own list."""
    img = synth.blob_field(41, 256, 256)
    if polarity == "dark":
        img = (1.0 - img).astype(np.float32)
    plan = fft_plan(max_hw=256, polarity=polarity)
    g = gpu_detect(plan, img)
    ora = oracle.log_stack(img, SIG10, polarity=0 if polarity == "bright" else 1)
    assert plane_rel_err(g["stack"], ora).max() <= FFT_TOL
    ykx, _ = oracle.candidates(ora, TAU)
    assert len(ykx) > 10
    plan_c = fft_plan(max_hw=256, polarity=polarity, overlap=1.0)
    g_c = gpu_detect(plan_c, img)
    compare_candidates(g_c["stack"], as_set(g_c["yxk"]), ora, as_set(ykx), TAU)
    keep = oracle.prune(g_c["yxk"], SIG10, 0.5)
    np.testing.assert_array_equal(g["yxk"], g_c["yxk"][keep])
    np.testing.assert_array_equal(g["resp"], g_c["resp"][keep])


def test_constant_image_has_no_response():
    img = np.full((128, 64), 0.6, np.float32)
    st = stack_of(fft_plan(max_hw=128), img)
    assert np.abs(st).max() <= FFT_TOL * 0.6


def test_whole_tile_4096_sampled_voxels():
    """A 4096 x 4096 8-bit tile (the longest transform): sampled voxels of
    every plane against the 2-D definition, and the whole stack against the
    direct path's (itself held to the oracle)."""
    from paper_2108_12050_amd import Plan
    img = synth.sem_tile(3, psf_sigma=1.0)
    t = torch.from_numpy(img).cuda()
    pf = fft_plan(max_hw=4096, dtype="u8", threshold=0.05)
    pd = Plan(sigmas=list(SIG10), threshold=0.05, overlap=0.5, dtype="u8", max_h=4096,
              max_w=4096)
    sf = pf.detect(t, return_stack=True).stack
    sd = pd.detect(t, return_stack=True).stack
    ref = sd.abs().amax(dim=(1, 2)).double()
    diff = (sf - sd).abs().amax(dim=(1, 2)).double() / ref
    assert float(diff.max()) <= 2 * FFT_TOL, diff
    I = oracle.to_f64(img)
    rng = np.random.default_rng(5)
    st = sf.cpu().numpy()
    for k, s in enumerate(SIG10):
        ys = np.r_[0, 4095, rng.integers(0, 4096, 10)]
        xs = np.r_[4095, 0, rng.integers(0, 4096, 10)]
        for y, x in zip(ys.tolist(), xs.tolist()):
            v = oracle.log_point(I, float(s), y, x)
            assert abs(st[k, y, x] - v) <= FFT_TOL * float(ref[k]), (k, y, x, st[k, y, x], v)


def test_refusals():
    from paper_2108_12050_amd import Plan
    plan = fft_plan(max_hw=256)
    with pytest.raises(_lib.MHFDError) as e:
        plan.detect(torch.zeros((100, 128), device=plan.device))
    assert e.value.status == 2
    for kw in (dict(max_h=8192), dict(stretch=True), dict(criterion="dog")):
        with pytest.raises(_lib.MHFDError):
            fft_plan(**kw)
    with pytest.raises(_lib.MHFDError):
        Plan(sigmas=[600.0], blur="fft", max_h=64, max_w=64)  # radius 2400 > 2048
    imgs = torch.zeros((1, 64, 64), device=plan.device)
    with pytest.raises(_lib.MHFDError):
        plan.focus_score(imgs, torch.tensor(SIG10, dtype=torch.float32, device=plan.device))
    from paper_2108_12050_amd.batch import detect_batched
    with pytest.raises(_lib.MHFDError):
        detect_batched(plan, [torch.zeros((64, 64), device=plan.device)])
