"""GPU parity of the soft focus score and its gradient (mhfd_focus_score,
mhfd_focus_score_backward through the C ABI) against the FP64 oracle.

Tolerances: scores within 1e-5 relative; sigma gradient within 1e-4 of its
largest component; image gradient element by element within 1e-4 of its
largest entry plus, per pixel, the bound of parity.kink_bound: at voxels whose
response lies within 1e-5 of the kink of |r| at 0 the sign of r, and with it
the cotangent, is decided by rounding on either side, and the bound is what
such a flip can move the image gradient.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import synth

from parity import kink_bound

pytestmark = pytest.mark.gpu

BETA, TAU = 50.0, 0.05


def make_plan(sig, h, w, sigma_cap=None):
    from paper_2108_12050_amd import Plan
    return Plan(sigmas=list(sig), max_h=h, max_w=w, sigma_cap=sigma_cap)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def min_abs_response(imgs, sig):
    return min(np.abs(oracle.log_stack(im, sig)).min() for im in imgs)


@pytest.mark.parametrize("shape,sig", [((2, 96, 80), [1.0, 2.0, 3.0, 4.5]),
                                       ((3, 70, 130), [1.5, 2.5, 6.0]),
                                       ((1, 33, 17), [1.0, 5.0])])
def test_forward_matches_oracle(shape, sig):
    B, H, W = shape
    imgs = np.stack([synth.blob_field(10 + b, H, W, n_blobs=max(2, H * W // 1300))
                     for b in range(B)])
    plan = make_plan(sig, H, W)
    s_gpu = plan.focus_score(to_dev(imgs), to_dev(np.float32(sig)), BETA, TAU).cpu().numpy()
    s_ora = oracle.soft_score(imgs.astype(np.float64), np.float64(np.float32(sig)), BETA, TAU)
    np.testing.assert_allclose(s_gpu, s_ora, rtol=1e-5, atol=0)


def test_constant_batch_closed_form():
    plan = make_plan([1.0, 2.0, 4.0], 64, 64)
    imgs = to_dev(np.full((2, 64, 50), 0.3))
    s = plan.focus_score(imgs, to_dev(np.float32([1.0, 2.0, 4.0])), BETA, TAU).cpu().numpy()
    # r = 0 exactly in real arithmetic; computed, it is the rounding of the
    # taps (FP16 pairs on the matrix cores: |r| <= 1e-7 of the image value),
    # which the softplus slope beta sigmoid(-beta tau) ~ 3.8 turns into
    # ~1e-6 of the score
    np.testing.assert_allclose(s, np.log1p(np.exp(-BETA * TAU)), rtol=4e-6)
    dI, ds = plan.focus_score_backward(imgs, to_dev(np.float32([1.0, 2.0, 4.0])),
                                       torch.ones(2, device="cuda"), BETA, TAU)
    # In exact arithmetic r = 0, so sgn(r) = 0 and both gradients vanish.  In
    # FP32 the taps sum to ~1e-8 rather than 0, r is rounding noise, and
    # sgn(noise) weights a sigma-derivative that is itself rounding noise:
    # bounds far below the gradients of real images (~1e-2).
    assert float(dI.abs().max()) < 1e-9 and float(ds.abs().max()) < 1e-6


def check_image_grad(dI, dI_o, imgs, sig, gbar):
    tol = 1e-4 * np.abs(dI_o).max()
    for b in range(len(imgs)):
        bound = kink_bound(imgs[b], sig, BETA, TAU, gbar[b])
        err = np.abs(dI[b] - dI_o[b])
        assert np.all(err <= tol + bound), (b, float((err - tol - bound).max()))
        assert (err > tol).mean() < 0.05   # flips stay local


@pytest.mark.parametrize("shape,sig", [((2, 64, 72), [1.0, 2.0, 3.0, 4.5]),
                                       ((1, 100, 61), [2.0, 3.0, 7.0]),
                                       ((2, 128, 128), [1.0, 2.0, 3.0, 4.0, 5.0])])
def test_backward_matches_oracle(shape, sig):
    B, H, W = shape
    sig32 = np.float32(sig)
    imgs = np.stack([synth.blob_field(20 + b, H, W, n_blobs=max(2, H * W // 1300))
                     for b in range(B)])
    gbar = np.float32(np.linspace(1.0, -0.5, B))
    plan = make_plan(sig, H, W)
    dI, ds = plan.focus_score_backward(to_dev(imgs), to_dev(sig32), to_dev(gbar), BETA, TAU)
    dI, ds = dI.cpu().numpy().astype(np.float64), ds.cpu().numpy().astype(np.float64)
    dI_o, ds_o = oracle.soft_score_grad(imgs.astype(np.float64), np.float64(sig32), BETA, TAU,
                                        gbar.astype(np.float64))
    np.testing.assert_allclose(ds, ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
    check_image_grad(dI, dI_o, imgs, np.float64(sig32), gbar)


def test_autograd_function():
    from paper_2108_12050_amd import focus_score
    H, W = 64, 64
    sig0 = [1.0, 2.0, 3.0]
    plan = make_plan(sig0, H, W, sigma_cap=5.0)
    imgs = to_dev(np.stack([synth.blob_field(3, H, W, n_blobs=5)])).requires_grad_(True)
    sig = to_dev(np.float32(sig0)).requires_grad_(True)
    s = focus_score(imgs, sig, plan, BETA, TAU)
    (2.0 * s.sum()).backward()
    dI, ds = plan.focus_score_backward(imgs.detach(), sig.detach(),
                                       torch.full((1,), 2.0, device="cuda"), BETA, TAU)
    assert torch.equal(imgs.grad, dI) and torch.equal(sig.grad, ds)
    # a few descent steps on the sigmas lower the score
    opt = torch.optim.SGD([sig], lr=0.5)
    first = None
    for _ in range(5):
        opt.zero_grad()
        loss = focus_score(imgs.detach(), sig, plan, BETA, TAU).sum()
        first = float(loss) if first is None else first
        loss.backward()
        opt.step()
    assert float(focus_score(imgs.detach(), sig.detach(), plan, BETA, TAU).sum()) < first


@pytest.mark.parametrize("factor", [1.13, 0.87])
def test_sigmas_off_the_plan_grid(factor):
    """Trainable sigmas away from the plan's: every call takes each scale's
    radius floor(4 sigma + 0.5) from the current sigma (here every radius
    differs from the plan's), so score and gradients equal the oracle's at
    those sigmas with their own radii."""
    B, H, W = 2, 90, 76
    grid = [1.0, 2.0, 3.0, 4.5]
    sig32 = np.float32(np.float32(grid) * np.float32(factor))
    sig = np.float64(sig32)
    assert all(oracle.radius(a) != oracle.radius(b) for a, b in zip(sig, grid))
    imgs = np.stack([synth.blob_field(40 + b, H, W, n_blobs=6) for b in range(B)])
    plan = make_plan(grid, H, W, sigma_cap=6.0)
    s_gpu = plan.focus_score(to_dev(imgs), to_dev(sig32), BETA, TAU).cpu().numpy()
    np.testing.assert_allclose(s_gpu, oracle.soft_score(imgs.astype(np.float64), sig, BETA, TAU),
                               rtol=1e-5, atol=0)
    gbar = np.float32([1.0, -0.75])
    dI, ds = plan.focus_score_backward(to_dev(imgs), to_dev(sig32), to_dev(gbar), BETA, TAU)
    dI, ds = dI.cpu().numpy().astype(np.float64), ds.cpu().numpy().astype(np.float64)
    dI_o, ds_o = oracle.soft_score_grad(imgs.astype(np.float64), sig, BETA, TAU,
                                        gbar.astype(np.float64))
    np.testing.assert_allclose(ds, ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
    check_image_grad(dI, dI_o, imgs, sig, gbar)


def test_sigma_crossing_a_radius_boundary():
    """Radius 9 below sigma = 2.375 and 10 above it: the scores on either
    side follow the oracle with the matching radius, and differ from each
    other by the truncation step, not by rounding."""
    H, W = 64, 80
    img = synth.blob_field(7, H, W, n_blobs=5)[None]
    plan = make_plan([1.0, 2.0, 3.0], H, W, sigma_cap=4.0)
    out = []
    for s2 in (2.37, 2.38):
        sig32 = np.float32([1.0, s2, 3.0])
        assert oracle.radius(float(sig32[1])) == (9 if s2 < 2.375 else 10)
        g = plan.focus_score(to_dev(img), to_dev(sig32), BETA, TAU).cpu().numpy()
        o = oracle.soft_score(img.astype(np.float64), np.float64(sig32), BETA, TAU)
        np.testing.assert_allclose(g, o, rtol=1e-5, atol=0)
        dI, ds = plan.focus_score_backward(to_dev(img), to_dev(sig32), to_dev(np.ones(1)),
                                           BETA, TAU)
        _, ds_o = oracle.soft_score_grad(img.astype(np.float64), np.float64(sig32), BETA, TAU)
        np.testing.assert_allclose(ds.cpu().numpy(), ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
        out.append(float(g[0]))
    assert out[0] != out[1]


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf"), 4.01])
def test_sigma_outside_the_cap_raises(bad):
    """A sigma outside (0, sigma_cap] sets the call's device error word; the
    binding raises on it.  The cap itself is accepted."""
    from paper_2108_12050_amd import MHFDError
    plan = make_plan([1.0, 2.0, 3.0], 40, 40, sigma_cap=4.0)
    img = to_dev(synth.blob_field(2, 40, 40, n_blobs=3)[None])
    plan.focus_score(img, to_dev(np.float32([1.0, 2.0, 4.0])), BETA, TAU)
    with pytest.raises(MHFDError):
        plan.focus_score(img, to_dev(np.float32([1.0, bad, 3.0])), BETA, TAU)
    with pytest.raises(MHFDError):
        plan.focus_score_backward(img, to_dev(np.float32([bad, 2.0, 3.0])), torch.ones(1).cuda(),
                                  BETA, TAU)
    plan.focus_score(img, to_dev(np.float32([1.0, 2.0, 3.0])), BETA, TAU)   # clears the word


def test_trained_sigmas_follow_the_oracle():
    """After SGD steps on the sigmas (which leave the plan's grid), score and
    sigma gradient at the trained sigmas equal the oracle's."""
    from paper_2108_12050_amd import focus_score
    H, W = 72, 72
    sig0 = [1.0, 2.0, 3.0]
    plan = make_plan(sig0, H, W, sigma_cap=5.0)
    img = np.stack([synth.blob_field(5, H, W, n_blobs=6)])
    t = to_dev(img)
    sig = to_dev(np.float32(sig0)).requires_grad_(True)
    for _ in range(4):   # normalised descent steps of 0.2 on the largest component
        sig.grad = None
        focus_score(t, sig, plan, BETA, TAU).sum().backward()
        with torch.no_grad():
            sig -= 0.2 * sig.grad / sig.grad.abs().max()
    s_now = np.float64(sig.detach().cpu().numpy())
    assert np.abs(s_now - sig0).max() > 0.05, s_now
    g = plan.focus_score(t, sig.detach(), BETA, TAU).cpu().numpy()
    np.testing.assert_allclose(g, oracle.soft_score(img.astype(np.float64), s_now, BETA, TAU),
                               rtol=1e-5, atol=0)
    _, ds = plan.focus_score_backward(t, sig.detach(), torch.ones(1).cuda(), BETA, TAU)
    _, ds_o = oracle.soft_score_grad(img.astype(np.float64), s_now, BETA, TAU)
    np.testing.assert_allclose(ds.cpu().numpy(), ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())


def test_full_size_gradient_batch():
    """8 x 2048 x 2048, sigma 1..10, beta 50, tau 0.05, the gradient workload:
    image 0 against the oracle (score, sigma gradient with gbar = e_0, image
    gradient along random directions); images with zero upstream gradient get
    an exactly zero image gradient."""
    B, H, W = 8, 2048, 2048
    print("full-size gradient batch", flush=True)
    imgs = synth.grad_batch(0, B, H, W)
    sig = np.float32(np.arange(1, 11))
    plan = make_plan(sig, H, W)
    t = to_dev(imgs)
    s_gpu = plan.focus_score(t, to_dev(sig), BETA, TAU).cpu().numpy()
    gbar = np.zeros(B, np.float32)
    gbar[0] = 1.0
    dI, ds = plan.focus_score_backward(t, to_dev(sig), to_dev(gbar), BETA, TAU)
    dI0 = dI[0].cpu().numpy().astype(np.float64)
    assert float(dI[1:].abs().max()) == 0.0
    ds = ds.cpu().numpy().astype(np.float64)
    print("oracle forward/backward on image 0", flush=True)
    I0 = imgs[0:1].astype(np.float64)
    s_ora = oracle.soft_score(I0, np.float64(sig), BETA, TAU)
    np.testing.assert_allclose(s_gpu[0], s_ora[0], rtol=1e-5)
    dI_o, ds_o = oracle.soft_score_grad(I0, np.float64(sig), BETA, TAU, np.ones(1))
    np.testing.assert_allclose(ds, ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
    check_image_grad(dI0[None], dI_o, imgs[0:1], np.float64(sig), [1.0])


def test_default_halos_follow_the_plan_radii():
    """Without sigma_cap each scale's halo is its plan radius rounded up to a
    multiple of 4: a sigma may move while its radius fits (scores then equal
    the oracle's at that sigma), and one whose radius outgrows it raises."""
    from paper_2108_12050_amd import MHFDError
    H, W = 60, 70
    img = synth.blob_field(8, H, W, n_blobs=5)[None]
    plan = make_plan([1.0, 2.0, 3.0], H, W)            # radii 4, 8, 12: halos 4, 8, 12
    sig32 = np.float32([1.1, 1.9, 3.12])                # radii 4, 8, 12
    g = plan.focus_score(to_dev(img), to_dev(sig32), BETA, TAU).cpu().numpy()
    np.testing.assert_allclose(g, oracle.soft_score(img.astype(np.float64), np.float64(sig32),
                                                    BETA, TAU), rtol=1e-5, atol=0)
    _, ds = plan.focus_score_backward(to_dev(img), to_dev(sig32), torch.ones(1).cuda(), BETA, TAU)
    _, ds_o = oracle.soft_score_grad(img.astype(np.float64), np.float64(sig32), BETA, TAU)
    np.testing.assert_allclose(ds.cpu().numpy(), ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
    with pytest.raises(MHFDError):   # radius 5 > halo 4
        plan.focus_score(to_dev(img), to_dev(np.float32([1.2, 2.0, 3.0])), BETA, TAU)


def test_vector_path_beyond_the_matrix_core_radius():
    """A sigma cap whose radius (60) exceeds the matrix cores' limit (56)
    sends every scale to the vector strip kernel with the same four tap sets:
    score, sigma gradient and image gradient against the oracle, at sigmas
    off the plan grid."""
    B, H, W = 2, 70, 66
    sig0 = [2.0, 5.0, 9.0]
    plan = make_plan(sig0, H, W, sigma_cap=15.0)
    sig32 = np.float32([2.3, 4.6, 9.7])
    imgs = np.stack([synth.blob_field(30 + b, H, W, n_blobs=5) for b in range(B)])
    gbar = np.float32([1.0, -0.7])
    g = plan.focus_score(to_dev(imgs), to_dev(sig32), BETA, TAU).cpu().numpy()
    np.testing.assert_allclose(g, oracle.soft_score(imgs.astype(np.float64), np.float64(sig32),
                                                    BETA, TAU), rtol=1e-5, atol=0)
    dI, ds = plan.focus_score_backward(to_dev(imgs), to_dev(sig32), to_dev(gbar), BETA, TAU)
    dI, ds = dI.cpu().numpy().astype(np.float64), ds.cpu().numpy().astype(np.float64)
    dI_o, ds_o = oracle.soft_score_grad(imgs.astype(np.float64), np.float64(sig32), BETA, TAU,
                                        gbar.astype(np.float64))
    np.testing.assert_allclose(ds, ds_o, rtol=0, atol=1e-4 * np.abs(ds_o).max())
    check_image_grad(dI, dI_o, imgs, np.float64(sig32), gbar)
