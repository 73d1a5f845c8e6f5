"""The serving scheduler on the CPU, with a host executor standing in for the
GPU: admission by HBM budget, arrival order, slot reuse and overlap,
rejection of requests that can never fit, and failures injected from the host
(a launch that raises, a batch whose tiles come back as errors)."""
import time

import numpy as np
import pytest

from paper_2108_12050_amd.serve import Request, Server


class HostExecutor:
    """Each slot finishes a batch after `latency_polls` polls; the result of a
    tile is a function of its pixels so that mix-ups are visible."""

    def __init__(self, n_slots=2, slot_tiles=4, slot_pixels=10_000, fixed_bytes=1000,
                 latency_polls=3, fail_launch=(), fail_tiles=(), fail_poll=(), flags=None):
        self.bytes_per_pixel = 4
        self.slot_tiles, self.slot_pixels, self.fixed_bytes = slot_tiles, slot_pixels, fixed_bytes
        self.latency_polls = latency_polls
        self.fail_launch, self.fail_tiles = set(fail_launch), set(fail_tiles)
        self.fail_poll, self.flags = set(fail_poll), dict(flags or {})
        self.completed = 0
        self.batches = [None] * n_slots
        self.polls = [0] * n_slots
        self.launches = 0
        self.staged = 0

    def stage(self, r):
        self.staged += 1
        return ("resident", r.rid)

    def idle_slots(self):
        return [i for i, b in enumerate(self.batches) if b is None]

    def launch(self, slot, batch):
        self.launches += 1
        if self.launches in self.fail_launch:
            raise RuntimeError("injected launch failure")
        assert all(r.staged == ("resident", r.rid) for r in batch)
        self.batches[slot] = batch
        self.polls[slot] = 0

    def poll(self, slot):
        self.polls[slot] += 1
        if self.polls[slot] < self.latency_polls:
            return None
        batch = self.batches[slot]
        self.batches[slot] = None
        self.completed += 1
        if self.completed in self.fail_poll:
            raise RuntimeError("injected read-back failure")
        return [RuntimeError("injected tile failure") if r.rid in self.fail_tiles
                else (int(np.asarray(r.image).sum()), r.pixels, self.flags.get(r.rid, 0),
                      1e6 * int(np.asarray(r.image).sum()) / r.pixels, None) for r in batch]


def img(h, w, v=1.0):
    return np.full((h, w), v, np.float32)


def test_serves_everything_in_order_within_budget():
    ex = HostExecutor()
    budget = ex.fixed_bytes + 4 * 2500   # room for 2500 pixels of tiles
    srv = Server(ex, budget)
    sizes = [(20, 30), (40, 40), (10, 10), (50, 40), (30, 30), (5, 7)] * 5
    for i, (h, w) in enumerate(sizes):
        assert srv.submit(Request(i, img(h, w, i % 3 + 1), time.perf_counter()))
    srv.drain(0.0)
    assert len(srv.finished) == len(sizes)
    for r in srv.finished:
        assert r.error is None and r.count == int(img(r.h, r.w, r.rid % 3 + 1).sum())
        assert r.admitted >= r.arrival and r.started >= r.admitted and r.done >= r.started
    assert srv.peak_resident + ex.fixed_bytes <= budget
    admitted_order = sorted(srv.finished, key=lambda r: r.admitted)
    assert [r.rid for r in admitted_order] == sorted(r.rid for r in srv.finished)
    assert srv.resident == 0 and not srv.busy()


def test_slots_overlap_and_are_reused():
    ex = HostExecutor(n_slots=2, slot_tiles=2, latency_polls=5)
    srv = Server(ex, 10**9)
    for i in range(12):
        srv.submit(Request(i, img(10, 10), time.perf_counter()))
    srv.drain(0.0)
    assert srv.max_inflight == 2
    assert ex.launches == 6   # 12 tiles, 2 per batch
    assert len(srv.finished) == 12


def test_tiny_budget_forces_queueing_but_serves_all():
    ex = HostExecutor(n_slots=2, slot_tiles=8)
    budget = ex.fixed_bytes + 4 * 100      # one 10x10 tile resident at a time
    srv = Server(ex, budget)
    for i in range(6):
        srv.submit(Request(i, img(10, 10), time.perf_counter()))
    srv.drain(0.0)
    assert len(srv.finished) == 6 and srv.peak_resident == 400
    assert srv.max_inflight == 1


def test_requests_that_can_never_fit_are_rejected():
    ex = HostExecutor(slot_pixels=1000)
    srv = Server(ex, ex.fixed_bytes + 4 * 500)
    assert not srv.submit(Request(0, img(40, 40), time.perf_counter()))   # > slot pixels
    assert not srv.submit(Request(1, img(25, 25), time.perf_counter()))   # > budget
    assert srv.submit(Request(2, img(10, 10), time.perf_counter()))
    srv.drain(0.0)
    assert [r.rid for r in srv.rejected] == [0, 1] and all(r.error for r in srv.rejected)
    assert [r.rid for r in srv.finished] == [2] and srv.finished[0].error is None


def test_injected_failures_do_not_stop_the_server():
    ex = HostExecutor(n_slots=1, slot_tiles=2, fail_launch={2}, fail_tiles={5})
    srv = Server(ex, 10**9)
    for i in range(8):
        srv.submit(Request(i, img(8, 8), time.perf_counter()))
    srv.drain(0.0)
    err = {r.rid: r.error for r in srv.finished}
    assert len(err) == 8
    assert err[2] and err[3] and "launch failed" in err[2]   # second batch failed to launch
    assert err[5] and "tile failure" in err[5]
    assert all(err[i] is None for i in (0, 1, 4, 6, 7))
    assert srv.resident == 0


def test_executor_workspace_larger_than_budget_is_refused():
    with pytest.raises(ValueError):
        Server(HostExecutor(fixed_bytes=5000), 4000)


def test_run_trace_real_time():
    ex = HostExecutor(latency_polls=2)
    srv = Server(ex, 10**9)
    arrivals = [0.0, 0.001, 0.002, 0.01, 0.011, 0.03]
    out = srv.run_trace(arrivals, [img(10, 10)] * len(arrivals), idle_sleep=0.0005)
    assert [r.rid for r in out] == list(range(6))
    assert all(r.error is None and r.latency >= 0 for r in out)
    assert all(r.arrival - out[0].arrival >= a - 1e-9 for r, a in zip(out, arrivals))


def test_read_back_failure_fails_its_batch_only():
    """A poll that raises (a device error surfacing when results are copied
    back) completes that batch's requests with the error; the server goes on."""
    ex = HostExecutor(n_slots=1, slot_tiles=2, fail_poll={2})
    srv = Server(ex, 10**9)
    for i in range(6):
        srv.submit(Request(i, img(8, 8), time.perf_counter()))
    srv.drain(0.0)
    err = {r.rid: r.error for r in srv.finished}
    assert len(err) == 6 and srv.resident == 0
    assert err[2] and err[3] and "read-back failure" in err[2]
    assert all(err[i] is None for i in (0, 1, 4, 5))


def test_flagged_results_are_errors():
    """Candidate overflow (flag 2) and an invalid tile (flag 4) make the
    request fail; a blob-list overflow (flag 1) keeps the valid count."""
    ex = HostExecutor(n_slots=1, slot_tiles=4, flags={1: 2, 2: 4, 3: 1})
    srv = Server(ex, 10**9)
    for i in range(4):
        srv.submit(Request(i, img(8, 8, 2.0), time.perf_counter()))
    srv.drain(0.0)
    r = {q.rid: q for q in srv.finished}
    assert r[0].error is None and r[0].count == 128 and r[0].density == 2e6
    assert r[1].error and "candidate" in r[1].error
    assert r[2].error and "invalid" in r[2].error
    assert r[3].error is None and r[3].flags == 1 and r[3].count == 128
    from paper_2108_12050_amd.serve import summarize
    assert summarize(srv.finished, 1.0)["served"] == 2
