"""The paper's own criterion (section 3: DoG of equation "dog", argmax over
scale and 3x3 maxpool equality of equation "argmax", the count of
Algorithm 1) on the GPU against the oracle.  The Gaussian planes the
matrix-core kernel writes are compared within 1e-5 of each plane's
maximum; the GPU's largest DoG is recomputed on the host from its planes in
the kernel's FP32 arithmetic, so its blob set and argmax are checked
exactly against that plane and, outside the ambiguity margin, against the
oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import synth

from parity import as_set, compare_candidates, own_maxima, plane_rel_err

pytestmark = pytest.mark.gpu

STACK_TOL = 1e-5
EPS = 1e-4


def dog_plan(max_hw, **kw):
    from paper_2108_12050_amd import Plan
    args = dict(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.01, overlap=1.0,
                max_h=max_hw, max_w=max_hw, criterion="dog")
    args.update(kw)
    return Plan(**args)


def gpu_dog_max(L32: np.ndarray, sig32: np.ndarray):
    """The DoG kernel's FP32 arithmetic: sig_i * (L_{i+1} - L_i), first max."""
    d = sig32[:-1, None, None] * (L32[1:] - L32[:-1])
    return d.max(axis=0), np.argmax(d, axis=0)


def check(plan, img, I, rows=None, row0=0, L_ora=None):
    tau = float(np.float32(plan.threshold))
    d = plan.detect(torch.from_numpy(img).to(plan.device), return_stack=True)
    L = d.stack.cpu().numpy()
    sig = np.asarray(plan.sigmas, np.float64)
    if L_ora is None:
        L_ora = oracle.gauss_stack(I, sig)
    a, b = (0, L.shape[1]) if rows is None else rows
    assert plane_rel_err(L[:, a:b], L_ora[:, a - row0:b - row0]).max() <= STACK_TOL
    M, arg = gpu_dog_max(L, np.asarray(plan.sigmas, np.float32))
    got = d.yxk.cpu().numpy()
    # records: exactly the maxpool-equality pixels of the GPU's own M plane,
    # labelled with its first argmax
    assert np.array_equal(got[:, 2], arg[got[:, 0], got[:, 1]])
    ora = oracle.dog_criterion(L_ora, sig, tau)
    g_set = {(y, x, 0) for y, x, _ in got.tolist()}
    o_set = {(y + row0, x, 0) for y, x, _ in ora["yxk"].tolist()}
    compare_candidates(M[None, row0:row0 + L_ora.shape[1]].astype(np.float32), g_set,
                       ora["M"][None], o_set, tau, rows=rows, row0=row0)
    # argmax against the oracle where the two best scales are apart
    dd = sig[:-1, None, None] * (L_ora[1:] - L_ora[:-1])
    srt = np.sort(dd, axis=0)
    clear = (srt[-1] - srt[-2]) > EPS
    ys, xs = got[:, 0] - row0, got[:, 1]
    inside = (ys >= 0) & (ys < L_ora.shape[1])
    ys, xs, ks = ys[inside], xs[inside], got[inside, 2]
    sel = clear[ys, xs]
    assert np.array_equal(ks[sel], ora["idx"][ys[sel], xs[sel]])
    return d, ora


@pytest.mark.parametrize("h,w", [(37, 23), (129, 200), (96, 300), (200, 264)])
def test_f32_dark_blobs(h, w):
    """Dark blobs on a bright background: the paper's DoG is positive there."""
    print(f"dog f32 {h}x{w}", flush=True)
    img = (1.0 - synth.blob_field(h * 3 + w, h, w, psf_sigma=1.0)).astype(np.float32)
    plan = dog_plan(512)
    d, ora = check(plan, img, img.astype(np.float64))
    if h * w > 10000:
        assert ora["count"] > 5


def test_u8_stretched_sem_tile():
    from paper_2108_12050_amd import Plan  # noqa: F401
    img = (255 - synth.sem_tile(6, psf_sigma=1.0, H=256, W=320)).astype(np.uint8)
    plan = dog_plan(512, dtype="u8", stretch=True, threshold=0.02)
    d, ora = check(plan, img, oracle.stretch(img))
    assert ora["count"] > 20


def test_full_size_u8_bands():
    """4096^2 SEM tile (inverted: dark texture), as a user would run the
    paper's criterion on it: over the whole tile, the blob list against the
    maxpool-equality rule on M recomputed from the GPU's planes; three row
    bands compared with the oracle run on the band plus a 42-row margin
    (rows y0 - 1 .. y1 of the planes are then exact)."""
    print("dog full-size 4096x4096 u8", flush=True)
    img = (255 - synth.sem_tile(2, psf_sigma=0.0)).astype(np.uint8)
    plan = dog_plan(4096, dtype="u8", threshold=0.02)
    I = oracle.to_f64(img)
    d = plan.detect(torch.from_numpy(img).to(plan.device), return_stack=True)
    L = d.stack.cpu().numpy()
    sig = np.asarray(plan.sigmas, np.float64)
    M, arg = gpu_dog_max(L, np.asarray(plan.sigmas, np.float32))
    got = d.yxk.cpu().numpy()
    assert np.array_equal(got[:, 2], arg[got[:, 0], got[:, 1]])
    g_set = {(y, x, 0) for y, x, _ in got.tolist()}
    tau = float(np.float32(0.02))
    own = own_maxima(M[None].astype(np.float32), tau)
    np.testing.assert_array_equal(got[:, :2].astype(np.int64), own[:, :2])
    m, H = 42, 4096
    for (y0, y1) in [(0, 96), (2000, 2096), (4000, 4096)]:
        a, b = max(0, y0 - m), min(H, y1 + m)
        L_ora = oracle.gauss_stack(I[a:b], sig)
        lo, hi = max(0, y0 - 1), min(H, y1 + 1)
        assert plane_rel_err(L[:, lo:hi], L_ora[:, lo - a:hi - a]).max() <= STACK_TOL
        ora = oracle.dog_criterion(L_ora, sig, tau)
        o_set = {(y + a, x, 0) for y, x, _ in ora["yxk"].tolist()}
        compare_candidates(M[None, a:b].astype(np.float32), g_set, ora["M"][None], o_set, tau,
                           rows=(y0, y1), row0=a)


def test_batched_and_focus_refuse_dog_plans():
    from paper_2108_12050_amd import MHFDError, detect_batched, focus_score
    plan = dog_plan(64)
    with pytest.raises(MHFDError):
        detect_batched(plan, [torch.zeros((32, 32), dtype=torch.float32, device="cuda")])
    with pytest.raises(MHFDError):
        focus_score(torch.zeros((1, 32, 32), dtype=torch.float32, device="cuda"),
                    torch.tensor(plan.sigmas, dtype=torch.float32, device="cuda"), plan)
