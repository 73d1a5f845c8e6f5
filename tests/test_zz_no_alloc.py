"""mhfd_log_stack_static, the entry point that allocates nothing (its scratch
is a static device array of the library), against mhfd_log_stack with a
caller workspace: identical stacks on two calls in a row, the second on a
smaller image whose scratch values differ from the first's (a larger fp32
range, another histogram), so a value left over from the first call would
show.  The stacks are also within 1e-5 of each plane's maximum of the
oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import Plan, _lib, synth

pytestmark = pytest.mark.gpu

SIG = oracle.linear_sigmas(10, 1.0, 10.0)


def run_both(plan, img: np.ndarray):
    L = _lib.load()
    t = torch.from_numpy(np.ascontiguousarray(img)).to(plan.device)
    h, w = t.shape
    s = int(torch.cuda.current_stream().cuda_stream)
    ref = torch.empty((plan.K, h, w), dtype=torch.float32, device=plan.device)
    got = torch.full_like(ref, float("nan"))
    n = L.mhfd_log_stack_workspace_size(plan._handle, h, w)
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=plan.device)
    _lib.check(L.mhfd_log_stack(plan._handle, t.data_ptr(), h, w, w, ref.data_ptr(),
                                ws.data_ptr(), n, s), "mhfd_log_stack")
    _lib.check(L.mhfd_log_stack_static(plan._handle, t.data_ptr(), h, w, w, got.data_ptr(), s),
               "mhfd_log_stack_static")
    torch.cuda.synchronize()
    return ref, got


def images(kind):
    if kind == "f32":
        big = (8.0 * synth.blob_field(1, 300, 260, n_blobs=40)).astype(np.float32)
        small = synth.blob_field(2, 120, 96, n_blobs=8)
        return big, small, big.astype(np.float64), small.astype(np.float64)
    big = synth.sem_tile(1, psf_sigma=1.0, H=300, W=264)
    small = (synth.sem_tile(2, psf_sigma=2.0, H=120, W=96) // 2 + 40).astype(np.uint8)
    if kind == "u8":
        return big, small, oracle.to_f64(big), oracle.to_f64(small)
    return big, small, oracle.stretch(big), oracle.stretch(small)


@pytest.mark.parametrize("kind", ["f32", "u8", "u8_stretch"])
def test_static_scratch_equals_workspace_call(kind):
    print(f"static scratch, {kind}", flush=True)
    plan = Plan(n_scales=10, sigma_min=1.0, sigma_max=10.0, threshold=0.05,
                dtype="f32" if kind == "f32" else "u8", stretch=kind == "u8_stretch",
                max_h=512, max_w=512)
    big, small, big64, small64 = images(kind)
    for img, I in ((big, big64), (small, small64)):
        ref, got = run_both(plan, img)
        assert torch.equal(ref, got), kind
        ora = oracle.log_stack(I, SIG)
        err = (np.abs(got.cpu().numpy() - ora).reshape(10, -1).max(1)
               / np.abs(ora).reshape(10, -1).max(1))
        assert err.max() <= 1e-5, err


def test_static_entry_point_checks_arguments():
    plan = Plan(n_scales=3, sigma_min=1.0, sigma_max=3.0, max_h=64, max_w=64)
    L = _lib.load()
    img = torch.zeros((32, 32), dtype=torch.float32, device=plan.device)
    out = torch.empty((3, 32, 32), dtype=torch.float32, device=plan.device)
    s = int(torch.cuda.current_stream().cuda_stream)
    assert L.mhfd_log_stack_static(plan._handle, img.data_ptr(), 65, 32, 32, out.data_ptr(), s) == 1
    assert L.mhfd_log_stack_static(plan._handle, img.data_ptr(), 32, 32, 32, None, s) == 1
    assert L.mhfd_log_stack_static(None, img.data_ptr(), 32, 32, 32, out.data_ptr(), s) == 1
