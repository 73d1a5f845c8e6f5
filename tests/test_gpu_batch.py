"""Batched detection (mhfd_detect_batched) against the single-tile path and
the oracle: identical per-tile results whatever the batch composition or
order, HIP-graph replay equal to eager execution, replay with new
descriptors without re-capture, and device-side rejection of bad
descriptors."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_12050_amd import synth

from parity import as_set, compare_candidates, own_maxima, strip_prune

pytestmark = pytest.mark.gpu

SIG10 = oracle.linear_sigmas(10, 1.0, 10.0)


def plan_f32(max_hw=1024, **kw):
    from paper_2108_12050_amd import Plan
    args = dict(n_scales=10, sigma_min=1.0, sigma_max=10.0, threshold=0.1, overlap=0.5,
                max_h=max_hw, max_w=max_hw)
    args.update(kw)
    return Plan(**args)


def small_mixed(seed, n, scale=0.125):
    tiles = synth.mixed_batch(seed, n, scale=scale)
    return [torch.from_numpy(t).cuda() for t in tiles]


def same(a, b):
    assert a.count == b.count and a.n_candidates == b.n_candidates, (a.count, b.count)
    assert torch.equal(a.yxk, b.yxk)
    assert torch.equal(a.sigma, b.sigma) and torch.equal(a.response, b.response)


def test_batched_equals_single_tile_path():
    from paper_2108_12050_amd import detect_batched
    plan = plan_f32()
    imgs = small_mixed(1, 12)
    got = detect_batched(plan, imgs)
    for im, g in zip(imgs, got):
        same(g, plan.detect(im))


def test_batched_against_oracle():
    from paper_2108_12050_amd import detect_batched
    plan_c = plan_f32(overlap=1.0)
    imgs = small_mixed(2, 6)
    got = detect_batched(plan_c, imgs)
    tau = float(np.float32(0.1))
    for im, g in zip(imgs, got):
        st = oracle.log_stack(im.cpu().numpy(), SIG10)
        ykx, _ = oracle.candidates(st, tau)
        d = plan_c.detect(im, return_stack=True)
        compare_candidates(d.stack.cpu().numpy(), as_set(g.yxk.cpu().numpy()), st, as_set(ykx), tau)


def test_order_and_composition_do_not_matter():
    from paper_2108_12050_amd import detect_batched
    plan = plan_f32()
    imgs = small_mixed(3, 9)
    ref = detect_batched(plan, imgs)
    perm = [4, 0, 8, 2, 7, 1, 6, 3, 5]
    got = detect_batched(plan, [imgs[i] for i in perm])
    for j, i in enumerate(perm):
        same(got[j], ref[i])
    sub = detect_batched(plan, [imgs[2], imgs[2], imgs[5]])   # repeated tile
    same(sub[0], ref[2])
    same(sub[1], ref[2])
    same(sub[2], ref[5])


def test_u8_batch_and_segment_override():
    from paper_2108_12050_amd import Plan, detect_batched
    plan = Plan(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, overlap=0.5, dtype="u8",
                max_h=700, max_w=700)
    imgs = [torch.from_numpy(synth.sem_tile(s, psf_sigma=p, H=h, W=w)).cuda()
            for s, p, h, w in [(1, 0.0, 300, 260), (2, 2.0, 700, 512), (3, 1.0, 64, 700)]]
    ref = [plan.detect(im) for im in imgs]
    for seg in ([0, 0, 0], [32, 64, 96], [512, 4096, 128]):
        got = detect_batched(plan, imgs, seg_rows=seg)
        for g, r in zip(got, ref):
            same(g, r)


def test_graph_replay_and_new_descriptors():
    from paper_2108_12050_amd import BatchRunner
    plan = plan_f32()
    a = small_mixed(4, 8)
    b = small_mixed(5, 8)
    px = max(sum(t.numel() for t in a), sum(t.numel() for t in b))
    r = BatchRunner(plan, 8, px, 1 << 14)
    r.set_tiles(a)
    g = r.capture()
    ref_a = [plan.detect(t) for t in a]
    ref_b = [plan.detect(t) for t in b]
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        for d, ref in zip(r.detections(), ref_a):
            same(d, ref)
        _ = plan.detect(a[rep])       # eager work between replays
    r.set_tiles(b)                    # new images and sizes, same graph
    g.replay()
    torch.cuda.synchronize()
    for d, ref in zip(r.detections(), ref_b):
        same(d, ref)


def test_invalid_descriptor_is_rejected_on_device():
    from paper_2108_12050_amd import BatchRunner, MHFDError
    plan = plan_f32(max_hw=256)
    imgs = [torch.rand(100, 90, device="cuda"), torch.rand(300, 50, device="cuda")]  # 300 > 256
    r = BatchRunner(plan, 2, 100 * 90 + 300 * 50, 1024)
    r.set_tiles(imgs)
    r.run()
    torch.cuda.synchronize()
    flags = r.results[:2, 2].cpu().numpy() & 0xFFFFFFFF
    assert np.all(flags & 4)
    with pytest.raises(MHFDError):
        r.detections()
    # exceeding the pixel bound is rejected the same way
    r2 = BatchRunner(plan, 2, 1000, 1024)
    r2.set_tiles([imgs[0]])
    r2.run()
    torch.cuda.synchronize()
    assert int(r2.results[0, 2]) & 4


def test_full_size_mixed_batch():
    """64 tiles with sizes drawn from {1024^2, 2048x1536, 3072x2048, 4096^2},
    the batched workload's shapes (8 distinct rendered images, one per size
    class and defocus pair, reused across the 64 descriptors): every tile equals
    the single-tile path, and for every distinct image the blob list is the
    candidate rule on the GPU's own stack followed by the oracle's prune."""
    from paper_2108_12050_amd import BatchRunner
    print("full-size mixed batch", flush=True)
    shapes = synth.mixed_batch_shapes(0, 64)
    pool = {}
    for i, (h, w, p) in enumerate(shapes):
        key = (h, w, i % 2)
        if key not in pool:
            pool[key] = torch.from_numpy(synth.blob_field(1000 + len(pool), h, w, psf_sigma=p)).cuda()
    imgs = [pool[(h, w, i % 2)] for i, (h, w, p) in enumerate(shapes)]
    plan = plan_f32(max_hw=4096)
    px = sum(t.numel() for t in imgs)
    r = BatchRunner(plan, 64, px, 1 << 17)
    r.set_tiles(imgs)
    r.run()
    got = r.detections()
    ref = {}
    for im, g in zip(imgs, got):
        k = im.data_ptr()
        if k not in ref:
            ref[k] = plan.detect(im)
        same(g, ref[k])
    plan_c = plan_f32(max_hw=4096, overlap=1.0)
    tau = float(np.float32(0.1))
    for im in {t.data_ptr(): t for t in imgs}.values():
        print(f"whole-tile rule {tuple(im.shape)}", flush=True)
        dc = plan_c.detect(im, return_stack=True)
        cand = dc.yxk.cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(cand, own_maxima(dc.stack.cpu().numpy(), tau))
        del dc
        kept = ref[im.data_ptr()].yxk.cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(kept, strip_prune(cand, SIG10, 0.5, int(im.shape[0])))


def test_u8_graph_replay_and_full_size_batch():
    """8-bit tiles through the persistent matrix-core LoG: a captured graph
    replayed with new descriptors equals the single-tile path, and 16 tiles
    of the 4096^2 SEM workload (4 rendered images reused) equal it too."""
    from paper_2108_12050_amd import BatchRunner, Plan
    print("u8 batch graph + full size", flush=True)
    plan = Plan(n_scales=10, sigma_min=1, sigma_max=10, threshold=0.05, overlap=0.5, dtype="u8",
                max_h=4096, max_w=4096)
    small_a = [torch.from_numpy(synth.sem_tile(s, psf_sigma=1.0, H=h, W=w)).cuda()
               for s, h, w in [(11, 512, 384), (12, 300, 640), (13, 96, 96)]]
    small_b = [torch.from_numpy(synth.sem_tile(s, psf_sigma=2.0, H=h, W=w)).cuda()
               for s, h, w in [(14, 640, 200), (15, 257, 333)]]
    px = max(sum(t.numel() for t in small_a), sum(t.numel() for t in small_b))
    r = BatchRunner(plan, 4, px, 1 << 15)
    r.set_tiles(small_a)
    g = r.capture()
    ref_a = [plan.detect(t) for t in small_a]
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        for d, ref in zip(r.detections(), ref_a):
            same(d, ref)
    r.set_tiles(small_b)
    g.replay()
    torch.cuda.synchronize()
    for d, t in zip(r.detections(), small_b):
        same(d, plan.detect(t))
    big = [torch.from_numpy(synth.sem_tile(0, psf_sigma=p)).cuda() for p in (0.0, 1.0, 2.0, 4.0)]
    imgs = [big[i % 4] for i in range(16)]
    rb = BatchRunner(plan, 16, 16 * 4096 * 4096, 1 << 17)
    rb.set_tiles(imgs)
    rb.run()
    got = rb.detections()
    ref = [plan.detect(t) for t in big]
    for i, d in enumerate(got):
        same(d, ref[i % 4])


@pytest.mark.parametrize("K", [10, 20])
def test_odd_shapes_and_one_column_lanes(K):
    """Odd widths (one column per maxima lane) and odd pixel counts (tile
    stack extents padded to whole float4s), and K = 20 (more than 16 scales:
    one column per lane at every width); widths around the 64-, 128- and
    256-column strips (two and four columns per lane at K = 10).  Every
    tile's list equals the single-tile path's."""
    from paper_2108_12050_amd import detect_batched
    plan = plan_f32(max_hw=520, n_scales=K)
    shapes = [(65, 63), (1, 1), (130, 129), (97, 128), (3, 257), (200, 66), (33, 191),
              (40, 260), (21, 516), (70, 254)]
    imgs = [torch.from_numpy(synth.blob_field(40 + i, h, w, psf_sigma=1.0)).cuda()
            for i, (h, w) in enumerate(shapes)]
    print(f"batch K={K} shapes {shapes}", flush=True)
    got = detect_batched(plan, imgs)
    for im, g in zip(imgs, got):
        same(g, plan.detect(im))
    assert sum(g.count for g in got) > 20


@pytest.mark.parametrize("lanes", [2, 3])
def test_lanes_equal_one_batch_and_replay(lanes):
    """Tiles dealt to concurrent sub-batches (lanes) give every tile the same
    result as the single-tile path, eagerly and from a captured graph
    replayed with new tiles of other sizes."""
    from paper_2108_12050_amd import BatchRunner
    plan = plan_f32()
    a = small_mixed(6, 8)
    b = small_mixed(7, 8)
    px = max(sum(t.numel() for t in a), sum(t.numel() for t in b))
    r = BatchRunner(plan, 8, px, 1 << 14, lanes=lanes)
    r.set_tiles(a)
    assert sum(r.lane_n) == 8 and all(n > 0 for n in r.lane_n)
    r.run()
    torch.cuda.synchronize()
    ref_a = [plan.detect(t) for t in a]
    for d, ref in zip(r.detections(), ref_a):
        same(d, ref)
    g = r.capture()
    ref_b = [plan.detect(t) for t in b]
    r.set_tiles(b)
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        for d, ref in zip(r.detections(), ref_b):
            same(d, ref)


def test_autotuner_choices_keep_results():
    """The autotuner picks a segment height per size class and a launch shape
    for a batch from its candidates; the tuned runner's results equal the
    single-tile path's (launch parameters change the time only)."""
    import os
    import tempfile
    from paper_2108_12050_amd.autotune import (BATCH_RULES, CANDIDATES, LANES, LOG_GROUPS,
                                               NMS_GROUPS, Autotuner)
    plan = plan_f32()
    imgs = small_mixed(9, 6)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        tuner = Autotuner(plan, path)
        classes = sorted(set(tuple(t.shape) for t in imgs))
        rep = tuner.tune(classes, reps=2)
        for c in classes:
            best, times = rep[c]
            assert best in CANDIDATES and 0 in times and times[best] <= min(times.values()) + 1e-9
        br = tuner.tune_batch_segments(imgs, reps=1)
        assert br["best"] in BATCH_RULES and set(br["times"]) == set(BATCH_RULES)
        assert br["times"][br["best"]] <= min(br["times"].values()) + 1e-9
        for t in imgs:
            sr = tuner.seg_rows_for(*t.shape)
            assert sr == 0 or (sr % 32 == 0 and 32 <= sr <= 4096)
        lt = tuner.tune_launch(imgs, reps=1)
        b = lt["best"]
        assert b["log_groups_per_cu"] in LOG_GROUPS and b["nms_groups_per_cu"] in NMS_GROUPS
        assert b["lanes"] in LANES and lt["best_ms"] <= lt["default_ms"] + 1e-9
        again = Autotuner(plan, path)          # the cache gives the same choices
        assert again.table == tuner.table and again.launch == tuner.launch
        assert again.batch_rule == tuner.batch_rule
        r = tuner.runner(len(imgs), sum(t.numel() for t in imgs), 1 << 14)
        r.set_tiles(imgs, [tuner.seg_rows_for(*t.shape) for t in imgs])
        r.run()
        torch.cuda.synchronize()
        for dd, t in zip(r.detections(), imgs):
            same(dd, plan.detect(t))


def test_batch_options_are_checked():
    import ctypes as C
    from paper_2108_12050_amd import _lib
    plan = plan_f32(max_hw=128)
    L = _lib.load()
    bad = _lib.BatchOpts(9, 8)
    assert L.mhfd_detect_batched(plan._handle, 1, 1 << 20, 100, C.byref(bad), 1 << 20, 1 << 20,
                                 None) == 1
