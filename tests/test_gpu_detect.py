"""GPU parity of the detector (mhfd_detect through the C ABI) against the
FP64 oracle on the same seeded inputs.

Tolerances: the LoG stack within 1e-5 of each plane's largest oracle value;
candidate and blob decisions identical wherever the oracle's decision is not
within 1e-4 of the threshold or of a window neighbour (ambiguous decisions
must be consistent with the GPU's own stack); blob lists bit-exact in
(y, x, k, sigma) whenever the candidate sets agree, with responses within the
stack tolerance.  Threshold and overlap are handed to the oracle as the
float32 values the plan holds.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2108_12050_amd import synth

from parity import (as_set, compare_candidates, gpu_detect, own_maxima, plane_rel_err,
                    strip_prune)

pytestmark = pytest.mark.gpu

SIG10 = oracle.linear_sigmas(10, 1.0, 10.0)
TAU = float(np.float32(0.1))
STACK_TOL = 1e-5
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def make_plan(**kw):
    from paper_2108_12050_amd import Plan
    args = dict(n_scales=10, sigma_min=1.0, sigma_max=10.0, threshold=0.1, overlap=0.5,
                max_h=1024, max_w=1024)
    args.update(kw)
    return Plan(**args)


@pytest.fixture(scope="module")
def plans():
    return dict(prune=make_plan(), cand=make_plan(overlap=1.0))


def test_plan_scales_match_paper_grid(plans):
    p = plans["prune"]
    np.testing.assert_array_equal(np.float64(p.sigmas), SIG10)
    assert p.radii == [oracle.radius(s, 4.0) for s in SIG10]
    from paper_2108_12050_amd import Plan
    q = Plan(n_scales=5, sigma_min=1.5, sigma_max=3.25, max_h=64, max_w=64)
    np.testing.assert_array_equal(np.float64(q.sigmas), oracle.linear_sigmas(5, 1.5, 3.25))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_plain_512_stack_and_blobs(plans, seed):
    print(f"plain 512x512 seed {seed}", flush=True)
    img = synth.plain_tile(seed)
    ora = oracle.detect(img, SIG10, 4.0, TAU, 0.5)
    g_c = gpu_detect(plans["cand"], img)
    err = plane_rel_err(g_c["stack"], ora["stack"])
    assert err.max() <= STACK_TOL, err
    n_amb, n_diff = compare_candidates(g_c["stack"], as_set(g_c["yxk"]), ora["stack"],
                                       as_set(ora["cand"]), TAU)
    assert g_c["n_cand"] == len(g_c["yxk"])
    g_p = gpu_detect(plans["prune"], img, return_stack=False)
    # The GPU's pruned list is the oracle's prune of the GPU's own candidates
    # (which agree with the oracle's at every unambiguous voxel, above).
    keep = oracle.prune(g_c["yxk"], SIG10, 0.5)
    np.testing.assert_array_equal(g_p["yxk"], g_c["yxk"][keep])
    np.testing.assert_array_equal(g_p["resp"], g_c["resp"][keep])
    np.testing.assert_array_equal(g_p["sigma"], np.float32(SIG10[g_c["yxk"][keep][:, 2]]))
    assert g_p["count"] == int(keep.sum()) and g_p["n_cand"] == len(g_c["yxk"])
    if n_diff == 0:
        np.testing.assert_array_equal(g_p["yxk"], ora["blobs"])
        np.testing.assert_allclose(g_p["resp"], ora["blob_resp"], rtol=0,
                                   atol=STACK_TOL * np.abs(ora["stack"]).max())
        assert g_p["count"] == ora["count"]
    print(f"seed {seed}: ambiguous {n_amb} differing {n_diff} blobs {g_p['count']}", flush=True)


def test_strict_seeds_bit_exact(plans):
    """Seeds with no decision within 1e-4 of the threshold or of a neighbour:
    the blob lists must be identical."""
    seeds = json.load(open(os.path.join(GOLD, "strict_seeds.json")))["seeds"]
    for s in seeds:
        print(f"strict seed {s}", flush=True)
        img = synth.blob_field(s, 256, 256)
        ora = oracle.detect(img, SIG10, 4.0, TAU, 0.5)
        g_c = gpu_detect(plans["cand"], img, return_stack=False)
        np.testing.assert_array_equal(g_c["yxk"], ora["cand"])
        g = gpu_detect(plans["prune"], img)
        assert plane_rel_err(g["stack"], ora["stack"]).max() <= STACK_TOL
        np.testing.assert_array_equal(g["yxk"], ora["blobs"])
        np.testing.assert_array_equal(g["sigma"], np.float32(ora["blob_sigma"]))
        np.testing.assert_allclose(g["resp"], ora["blob_resp"], rtol=0,
                                   atol=STACK_TOL * np.abs(ora["stack"]).max())
        assert g["count"] == ora["count"] > 20


@pytest.mark.parametrize("shape", [(1, 1), (3, 2), (5, 70), (70, 5), (33, 65), (97, 130),
                                   (200, 129), (64, 64)])
def test_ragged_and_tiny_shapes(shape):
    """Kernel radius larger than the image, widths and heights that are not
    multiples of the strip width (64) or chunk height (32)."""
    print(f"shape {shape}", flush=True)
    rng = np.random.default_rng(sum(shape))
    img = synth.blob_field(5, *shape, n_blobs=max(1, shape[0] * shape[1] // 500)) \
        + rng.uniform(0, 0.05, shape).astype(np.float32)
    plan = make_plan(overlap=1.0, max_h=256, max_w=256)
    g = gpu_detect(plan, img)
    ora = oracle.log_stack(img, SIG10)
    err = np.abs(g["stack"] - ora).max()
    assert err <= STACK_TOL * max(np.abs(ora).max(), np.abs(img).max()), err
    ykx, _ = oracle.candidates(ora, TAU)
    compare_candidates(g["stack"], as_set(g["yxk"]), ora, as_set(ykx), TAU)


def test_constant_image_has_no_response():
    plan = make_plan(max_h=128, max_w=128)
    img = np.full((100, 77), 0.6, np.float32)
    g = gpu_detect(plan, img)
    assert np.abs(g["stack"]).max() < 1e-6
    assert g["count"] == 0 and g["n_cand"] == 0


def test_u8_input_and_pitch():
    """8-bit input read as u/255, from a row-padded buffer (pitch > width)."""
    import torch
    from paper_2108_12050_amd import Plan
    img = synth.sem_tile(1, psf_sigma=1.0, H=300, W=260)
    plan = Plan(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, overlap=0.5,
                dtype="u8", max_h=512, max_w=512)
    big = np.zeros((300, 300), np.uint8)
    big[:, :260] = img
    plan_c = Plan(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, overlap=1.0,
                  dtype="u8", max_h=512, max_w=512)
    t = torch.from_numpy(big).to(plan.device)[:, :260]
    assert t.stride(0) == 300
    tau = float(np.float32(0.05))
    d = plan.detect(t, return_stack=True)
    dc = plan_c.detect(t, return_stack=True)
    ora = oracle.detect(img, SIG10, 4.0, tau, 0.5)
    st = dc.stack.cpu().numpy()
    assert torch.equal(d.stack, dc.stack)
    assert plane_rel_err(st, ora["stack"]).max() <= STACK_TOL
    cand = dc.yxk.cpu().numpy().astype(np.int64)
    n_amb, n_diff = compare_candidates(st, as_set(cand), ora["stack"], as_set(ora["cand"]), tau)
    keep = oracle.prune(cand, SIG10, 0.5)
    np.testing.assert_array_equal(d.yxk.cpu().numpy().astype(np.int64), cand[keep])
    assert d.count == int(keep.sum()) and d.n_candidates == len(cand)
    if n_diff == 0:
        np.testing.assert_array_equal(cand[keep], ora["blobs"])
    print(f"u8 pitch: ambiguous {n_amb} differing {n_diff} blobs {d.count}", flush=True)


def test_dark_polarity_and_scale_grid():
    plan = make_plan(n_scales=4, sigma_min=1.5, sigma_max=3.0, polarity="dark", overlap=1.0,
                     max_h=128, max_w=128)
    sig = oracle.linear_sigmas(4, 1.5, 3.0)
    img = 1.0 - synth.blob_field(9, 128, 96, n_blobs=12)
    g = gpu_detect(plan, img)
    ora = oracle.log_stack(img, sig, polarity=1)
    assert plane_rel_err(g["stack"], ora).max() <= STACK_TOL
    ykx, _ = oracle.candidates(ora, TAU)
    compare_candidates(g["stack"], as_set(g["yxk"]), ora, as_set(ykx), TAU)
    assert len(ykx) > 3


def test_single_scale():
    plan = make_plan(n_scales=1, sigma_min=2.0, sigma_max=2.0, overlap=1.0, max_h=64, max_w=64)
    img = synth.blob_field(3, 64, 64, n_blobs=6)
    g = gpu_detect(plan, img)
    ora = oracle.log_stack(img, [2.0])
    assert plane_rel_err(g["stack"], ora).max() <= STACK_TOL
    ykx, _ = oracle.candidates(ora, TAU)
    compare_candidates(g["stack"], as_set(g["yxk"]), ora, as_set(ykx), TAU)


@pytest.mark.parametrize("K,w", [(3, 300), (4, 516), (2, 260), (7, 372), (10, 516)])
def test_four_columns_per_lane(K, w):
    """Up to ten planes the maxima pass reads four columns per lane (strips of
    256 columns, a 64-bit hit mask beyond 32 (column, plane) pairs): widths
    past one strip, with a ragged last strip."""
    plan = make_plan(n_scales=K, sigma_min=1.5, sigma_max=3.5, overlap=1.0, max_h=160,
                     max_w=520)
    sig = oracle.linear_sigmas(K, 1.5, 3.5)
    img = synth.blob_field(20 + K, 150, w, n_blobs=60)
    g = gpu_detect(plan, img)
    ora = oracle.log_stack(img, sig)
    assert plane_rel_err(g["stack"], ora).max() <= STACK_TOL
    ykx, _ = oracle.candidates(ora, TAU)
    compare_candidates(g["stack"], as_set(g["yxk"]), ora, as_set(ykx), TAU)
    assert len(ykx) > 10


def test_capacity_overflow_truncates_in_canonical_order(plans):
    img = synth.plain_tile(0)
    full = gpu_detect(plans["prune"], img, return_stack=False)
    part = gpu_detect(plans["prune"], img, return_stack=False, capacity=7)
    assert part["count"] == full["count"] > 7
    assert part["flags"] & 1
    np.testing.assert_array_equal(part["yxk"], full["yxk"][:7])


def test_deterministic(plans):
    img = synth.plain_tile(4)
    a = gpu_detect(plans["prune"], img)
    b = gpu_detect(plans["prune"], img)
    np.testing.assert_array_equal(a["stack"], b["stack"])
    np.testing.assert_array_equal(a["yxk"], b["yxk"])
    np.testing.assert_array_equal(a["resp"], b["resp"])


def test_errors_are_reported():
    import torch
    from paper_2108_12050_amd import MHFDError
    plan = make_plan(max_h=64, max_w=64)
    with pytest.raises(MHFDError):
        plan.detect(torch.zeros((65, 10), device=plan.device))
    with pytest.raises(MHFDError):
        make_plan(sigmas=[2.0, 1.0])
    with pytest.raises(MHFDError):
        make_plan(n_scales=1, sigma_min=20.0, sigma_max=20.0)   # radius 80 > 64


def test_split_entry_points_equal_detect(plans):
    """mhfd_log_stack followed by mhfd_detect_stack gives what mhfd_detect gives."""
    import torch
    from paper_2108_12050_amd import _lib
    p = plans["prune"]
    L = _lib.load()
    img = torch.from_numpy(synth.plain_tile(6)).to(p.device)
    d = p.detect(img, return_stack=True)
    st = torch.empty_like(d.stack)
    s = int(torch.cuda.current_stream().cuda_stream)
    nl = L.mhfd_log_stack_workspace_size(p._handle, 512, 512)
    lws = torch.empty(max(nl, 1), dtype=torch.uint8, device=p.device)
    _lib.check(L.mhfd_log_stack(p._handle, img.data_ptr(), 512, 512, 512, st.data_ptr(),
                                lws.data_ptr(), nl, s), "ls")
    cap = 4096
    raw = torch.empty((cap, 5), dtype=torch.int32, device=p.device)
    res = torch.zeros(_lib.RESULT_WORDS, dtype=torch.int64, device=p.device)
    nb = p.detect_workspace_bytes(512, 512)
    ws = torch.empty(nb, dtype=torch.uint8, device=p.device)
    _lib.check(L.mhfd_detect_stack(p._handle, st.data_ptr(), 512, 512, raw.data_ptr(), cap,
                                   res.data_ptr(), ws.data_ptr(), nb, s), "ds")
    torch.cuda.synchronize()
    assert torch.equal(st, d.stack)
    n = int(res[0])
    assert n == d.count
    assert torch.equal(raw[:n, :3], d.yxk)
    # the threshold-sparse halves give what mhfd_detect without a stack gives
    na = L.mhfd_activity_bytes(p._handle, 512, 512)
    assert na == 8 * 10 * 32 * 32
    act = torch.empty(na // 8, dtype=torch.int64, device=p.device)
    sp = torch.full_like(st, float("nan"))
    _lib.check(L.mhfd_log_stack_sparse(p._handle, img.data_ptr(), 512, 512, 512, sp.data_ptr(),
                                       act.data_ptr(), lws.data_ptr(), nl, s), "lss")
    res2 = torch.zeros(_lib.RESULT_WORDS, dtype=torch.int64, device=p.device)
    raw2 = torch.empty((cap, 5), dtype=torch.int32, device=p.device)
    _lib.check(L.mhfd_detect_stack_sparse(p._handle, sp.data_ptr(), act.data_ptr(), 512, 512,
                                          raw2.data_ptr(), cap, res2.data_ptr(), ws.data_ptr(),
                                          nb, s), "dss")
    d2 = p.detect(img)
    torch.cuda.synchronize()
    assert int(res2[0]) == d2.count == n and int(res2[1]) == d2.n_candidates
    assert torch.equal(raw2[:n], raw[:n])
    # written groups hold the dense stack's values, and every value above the
    # threshold lies in a written group
    bits = act.cpu().numpy().view(np.uint64).reshape(10, 32, 32)
    g = np.zeros((10, 512, 128), bool)
    for r in range(16):
        for q in range(4):
            g[:, r::16, q::4] = ((bits >> np.uint64(16 * q + r)) & np.uint64(1)).astype(bool)
    full = np.repeat(g, 4, axis=2)
    dense, spv = st.cpu().numpy(), sp.cpu().numpy()
    np.testing.assert_array_equal(spv[full], dense[full])
    assert not np.any(dense[~full] > np.float32(0.1))
    assert np.all(np.isnan(spv[~full])) and 0.02 < full.mean() < 0.6


def test_full_size_sem_tile():
    """4096 x 4096 8-bit tile, sigma 1..10, threshold 0.05, in the launch
    configuration the benchmark times, against one whole-tile oracle run:
    every voxel of the stack within 1e-5 of its plane's maximum, every
    candidate decision equal to the oracle's outside the ambiguity margin
    (ambiguous ones consistent with the GPU's own stack), the whole candidate
    list equal to the candidate rule on the GPU's own stack, and the pruned
    list equal to the oracle's prune of the GPU's candidates (and to the
    oracle's own list when no decision differs)."""
    import torch
    from paper_2108_12050_amd import Plan
    print("full-size 4096x4096 u8", flush=True)
    img = synth.sem_tile(0, psf_sigma=0.0)
    tau = float(np.float32(0.05))
    kw = dict(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, dtype="u8",
              max_h=4096, max_w=4096)
    plan_c, plan_p = Plan(overlap=1.0, **kw), Plan(overlap=0.5, **kw)
    t = torch.from_numpy(img).to(plan_c.device)
    d = plan_c.detect(t, return_stack=True)
    st = d.stack.cpu().numpy()
    d.stack = None
    cand = d.yxk.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(cand, own_maxima(st, tau))
    kept = plan_p.detect(t).yxk.cpu().numpy().astype(np.int64)
    print("oracle stack, whole tile", flush=True)
    ora = oracle.log_stack(oracle.to_f64(img), SIG10)
    err = plane_rel_err(st, ora)
    print(f"stack: largest plane error {err.max():.2e}", flush=True)
    assert err.max() <= STACK_TOL, err
    ykx, _ = oracle.candidates(ora, tau)
    n_amb, n_diff = compare_candidates(st, as_set(cand), ora, as_set(ykx), tau)
    print(f"candidates gpu {len(cand)} oracle {len(ykx)} ambiguous {n_amb} differing {n_diff}",
          flush=True)
    del ora, st
    np.testing.assert_array_equal(kept, strip_prune(cand, SIG10, 0.5, 4096))
    if n_diff == 0:
        np.testing.assert_array_equal(kept, strip_prune(ykx.astype(np.int64), SIG10, 0.5, 4096))
    assert len(kept) > 1000


def test_max_size_f32_tile():
    """8192 x 8192 fp32 tile (the largest size served), rendered like the
    plain workload (51200 blobs), sigma 1..10, threshold 0.1: sampled stack
    voxels against the 2-D definition; the whole candidate list against the
    candidate rule on the GPU's own stack; stack and candidate decisions
    (ambiguity-aware) against the oracle on three full-width row bands; and
    the overlap prune exactly, over the whole tile: a blob's fate depends only
    on candidates within r_a + r_b <= 2 sqrt(2) sigma_max of it, so the GPU's
    own candidate set, cut into 128-row strips with a 32-row margin, goes
    through the oracle's prune and must give the GPU's pruned list."""
    import torch
    print("max-size 8192x8192 f32", flush=True)
    H = W = 8192
    img = synth.blob_field(5, H, W)
    plan_c = make_plan(overlap=1.0, max_h=H, max_w=W)
    plan_p = make_plan(max_h=H, max_w=W)
    t = torch.from_numpy(img).to(plan_c.device)
    d = plan_c.detect(t, return_stack=True)
    cand = d.yxk.cpu().numpy().astype(np.int64)
    assert d.n_candidates == len(cand) and d.count == len(cand)
    np.testing.assert_array_equal(cand, own_maxima(d.stack.cpu().numpy(), TAU))
    I = oracle.to_f64(img)
    rng = np.random.default_rng(1)
    pts = [(int(rng.integers(0, 10)), int(rng.integers(0, H)), int(rng.integers(0, W)))
           for _ in range(200)]
    pts += [(k, y, x) for k in (0, 9) for y in (0, H - 1) for x in (0, 64, W - 1)]
    idx = torch.tensor(pts, dtype=torch.long, device=d.stack.device)
    vals = d.stack[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    for (k, y, x), v in zip(pts, vals):
        ref = oracle.log_point(I, SIG10[k], y, x)
        assert abs(v - ref) <= STACK_TOL * 0.5, (k, y, x, v, ref)
    m = 42   # > largest radius + 1: band rows [y0 - 1, y1 + 1) are exact
    gpu_c = as_set(cand)
    for (y0, y1) in [(0, 96), (4000, 4096), (H - 96, H)]:
        a, b = max(0, y0 - m), min(H, y1 + m)
        st = d.stack[:, a:b].cpu().numpy()
        ora = oracle.log_stack(I[a:b], SIG10)
        lo, hi = max(0, y0 - 1) - a, min(H, y1 + 1) - a
        err = plane_rel_err(st[:, lo:hi], ora[:, lo:hi])
        assert err.max() <= STACK_TOL, err
        ykx, _ = oracle.candidates(ora, TAU)
        ykx[:, 0] += a
        n_amb, n_diff = compare_candidates(st, gpu_c, ora, as_set(ykx), TAU,
                                           rows=(y0, y1), row0=a)
        print(f"band {y0}-{y1}: ambiguous {n_amb} differing {n_diff}", flush=True)
    del d, t
    dp = plan_p.detect(torch.from_numpy(img).to(plan_p.device))
    assert dp.n_candidates == len(cand)
    kept = dp.yxk.cpu().numpy().astype(np.int64)
    assert dp.count == len(kept)
    assert 2 * np.sqrt(2) * SIG10[-1] < 32
    expect = strip_prune(cand, SIG10, 0.5, H)
    print(f"candidates {len(cand)} kept {len(kept)}", flush=True)
    np.testing.assert_array_equal(kept, expect)
    assert 0 < len(kept) < len(cand)


def test_benchmark_tiles_prune_and_focus_order():
    """The benchmark's four 4096 x 4096 8-bit tiles (one scene, PSF sigma 0, 1,
    2, 4), threshold 0.05, overlap 0.5, in its launch configuration: sampled
    stack voxels against the 2-D definition, the prune exactly over each whole
    tile (the GPU's candidates through the oracle's prune, strip by strip),
    and the focus criterion's order: fewer blobs as the defocus grows."""
    import torch
    from paper_2108_12050_amd import Plan, detect_batched
    kw = dict(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, dtype="u8",
              max_h=4096, max_w=4096)
    plan_c, plan_p = Plan(overlap=1.0, **kw), Plan(overlap=0.5, **kw)
    counts, tiles, expected = [], [], []
    for psf in (0.0, 1.0, 2.0, 4.0):
        print(f"benchmark tile psf {psf}", flush=True)
        img = synth.sem_tile(0, psf_sigma=psf)
        t = torch.from_numpy(img).to(plan_c.device)
        d = plan_c.detect(t, return_stack=True)
        cand = d.yxk.cpu().numpy().astype(np.int64)
        I = oracle.to_f64(img)
        rng = np.random.default_rng(int(psf))
        pts = [(int(rng.integers(0, 10)), int(rng.integers(0, 4096)),
                int(rng.integers(0, 4096))) for _ in range(60)]
        idx = torch.tensor(pts, dtype=torch.long, device=d.stack.device)
        vals = d.stack[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
        for (k, y, x), v in zip(pts, vals):
            ref = oracle.log_point(I, SIG10[k], y, x)
            assert abs(v - ref) <= STACK_TOL * 0.5, (psf, k, y, x, v, ref)
        del d
        dp = plan_p.detect(t)
        kept = dp.yxk.cpu().numpy().astype(np.int64)
        assert dp.n_candidates == len(cand) and dp.count == len(kept)
        exp = strip_prune(cand, SIG10, 0.5, 4096)
        np.testing.assert_array_equal(kept, exp)
        print(f"psf {psf}: candidates {len(cand)} kept {len(kept)}", flush=True)
        counts.append(len(kept))
        tiles.append(t)
        expected.append(exp)
    assert counts == sorted(counts, reverse=True) and counts[-1] < counts[0] / 2, counts
    print("batched, the same four tiles", flush=True)
    for dt, exp in zip(detect_batched(plan_p, tiles, capacity=1 << 17), expected):
        np.testing.assert_array_equal(dt.yxk.cpu().numpy().astype(np.int64), exp)


@pytest.mark.parametrize("dtype,shape,K,seed", [("f32", (512, 512), 10, 0), ("f32", (97, 130), 10, 1),
                                                ("f32", (200, 129), 4, 2), ("u8", (300, 260), 10, 3),
                                                ("u8", (33, 65), 10, 4), ("u8", (1, 50), 3, 5),
                                                ("f32", (64, 64), 1, 6), ("u8", (1000, 1000), 10, 7)])
def test_threshold_sparse_stack_equals_dense(dtype, shape, K, seed):
    """Without a caller stack the detector writes and reads only the 4-pixel
    groups above the threshold; with one it writes the whole stack.  Both
    must give the same candidates, responses, blobs and counts (values at or
    below the threshold can neither be candidates nor block one)."""
    import torch
    from paper_2108_12050_amd import Plan
    print(f"sparse vs dense {dtype} {shape} K={K}", flush=True)
    H, W = shape
    if dtype == "u8":
        img = synth.sem_tile(seed, psf_sigma=1.0, H=H, W=W)
        tau = 0.05
    else:
        img = synth.blob_field(seed, H, W, n_blobs=max(1, H * W // 1300))
        tau = 0.1
    for overlap in (1.0, 0.5):
        plan = Plan(n_scales=K, sigma_min=1.0, sigma_max=max(1.0, K * 1.0), threshold=tau,
                    overlap=overlap, dtype=dtype, max_h=1024, max_w=1024)
        t = torch.from_numpy(img).to(plan.device)
        dense = plan.detect(t, return_stack=True)
        sparse = plan.detect(t)
        assert torch.equal(dense.yxk, sparse.yxk)
        assert torch.equal(dense.response, sparse.response)
        assert (dense.count, dense.n_candidates) == (sparse.count, sparse.n_candidates)
        own = own_maxima(dense.stack.cpu().numpy(), tau)
        if overlap >= 1.0:
            np.testing.assert_array_equal(sparse.yxk.cpu().numpy().astype(np.int64), own)


def test_threshold_sparse_dark_polarity_and_stretch():
    import torch
    from paper_2108_12050_amd import Plan
    img = 1.0 - synth.blob_field(9, 160, 200, n_blobs=20)
    plan = Plan(n_scales=6, sigma_min=1.0, sigma_max=6.0, polarity="dark", threshold=0.1,
                overlap=0.5, max_h=256, max_w=256)
    t = torch.from_numpy(img).to(plan.device)
    a, b = plan.detect(t, return_stack=True), plan.detect(t)
    assert torch.equal(a.yxk, b.yxk) and a.count == b.count > 3
    u8 = synth.sem_tile(2, psf_sigma=0.0, H=256, W=320)
    plan = Plan(n_scales=10, sigma_min=1.0, sigma_max=10.0, threshold=0.05, overlap=0.5,
                dtype="u8", stretch=True, max_h=256, max_w=320)
    t = torch.from_numpy(u8).to(plan.device)
    a, b = plan.detect(t, return_stack=True), plan.detect(t)
    assert torch.equal(a.yxk, b.yxk) and torch.equal(a.response, b.response) and a.count > 10
