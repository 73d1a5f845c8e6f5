"""Continuous-batching focus-detection server on one GPU.

Requests (one tile each) arrive at any time.  Each scheduler iteration:

  1. completes finished batches (results copied out, the tiles' device
     memory released); a batch whose execution or read-back raised, and a
     tile whose result carries the candidate-overflow or invalid-tile flag,
     complete with an error instead, and the loop goes on;
  2. admits waiting requests in arrival order while the HBM budget allows:
     the budget is charged the executor's fixed workspaces once and every
     admitted tile while it is resident; an admitted tile's host-to-device
     copy starts at once;
  3. launches a batch on every idle slot with the admitted tiles that fit its
     tile and pixel bounds -- so a batch formed from late arrivals runs while
     an earlier one is still on the device.

The scheduler only talks to an executor: `GpuExecutor` runs batches with
mhfd_detect_batched on per-slot streams (plans, workspaces, descriptor
tables and outputs stay on the device for the server's lifetime); tests use
a host executor to exercise admission, ordering and failures without a GPU.
Latency is arrival to result on the host, host-to-device copy included.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

FLAG_CAND_OVERFLOW = 2   # mhfd_result flags (include/mhfd.h)
FLAG_INVALID_TILE = 4


@dataclass
class Request:
    rid: int
    image: object                # host image (a pinned torch tensor for the GPU executor)
    arrival: float               # time.perf_counter() seconds
    h: int = 0
    w: int = 0
    staged: object = None        # executor's handle of the resident copy
    admitted: float = 0.0
    started: float = 0.0
    done: float = 0.0
    count: int = -1
    n_candidates: int = -1
    flags: int = 0
    density: float = 0.0
    device_ms: float = -1.0      # the request's batch on the device (start to end)
    blobs: np.ndarray | None = None
    error: str | None = None

    def __post_init__(self):
        if not self.h:
            self.h, self.w = int(self.image.shape[0]), int(self.image.shape[1])

    @property
    def pixels(self) -> int:
        return self.h * self.w

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Admission by HBM budget and continuous batching over an executor's
    slots (each slot runs one batch of up to `tiles` tiles / `pixels`
    pixels at a time)."""

    def __init__(self, executor, hbm_budget: int):
        self.ex = executor
        if executor.fixed_bytes > hbm_budget:
            raise ValueError(f"executor workspaces need {executor.fixed_bytes} bytes, budget "
                             f"{hbm_budget}")
        self.budget = hbm_budget
        self.resident = 0
        self.waiting: collections.deque[Request] = collections.deque()
        self.admitted: collections.deque[Request] = collections.deque()
        self.running: dict[int, list[Request]] = {}
        self.finished: list[Request] = []
        self.rejected: list[Request] = []
        self.peak_resident = 0
        self.max_inflight = 0

    def tile_bytes(self, r: Request) -> int:
        return r.pixels * self.ex.bytes_per_pixel

    def submit(self, req: Request) -> bool:
        """Queue a request; one that can never fit a slot or the budget is
        rejected at once (returns False, req.error set)."""
        if req.pixels > self.ex.slot_pixels:
            req.error = f"{req.pixels} pixels exceed a slot's {self.ex.slot_pixels}"
        elif self.ex.fixed_bytes + self.tile_bytes(req) > self.budget:
            req.error = "the tile can never fit the HBM budget"
        if req.error:
            req.done = time.perf_counter()
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def busy(self) -> bool:
        return bool(self.waiting or self.admitted or self.running)

    def _complete(self) -> None:
        for slot, batch in list(self.running.items()):
            try:
                out = self.ex.poll(slot)
            except Exception as e:  # read-back failed: the batch fails, the server goes on
                out = [e] * len(batch)
            if out is None:
                continue
            now = time.perf_counter()
            for r, res in zip(batch, out):
                if isinstance(res, Exception):
                    r.error = f"batch failed: {res}"
                else:
                    r.count, r.n_candidates, r.flags, r.density, r.blobs = res[:5]
                    if len(res) > 5:
                        r.device_ms = res[5]
                    if r.flags & FLAG_CAND_OVERFLOW:
                        r.error = (f"{r.n_candidates} candidates exceed the plan's candidate "
                                   "capacity: the count and list are not valid")
                    elif r.flags & FLAG_INVALID_TILE:
                        r.error = "invalid tile: the descriptor failed the device-side checks"

                r.done = now
                r.staged = None
                self.resident -= self.tile_bytes(r)
                self.finished.append(r)
            del self.running[slot]

    def _admit(self) -> None:
        while self.waiting:
            r = self.waiting[0]
            need = self.tile_bytes(r)
            if self.ex.fixed_bytes + self.resident + need > self.budget:
                break
            self.waiting.popleft()
            r.staged = self.ex.stage(r)
            r.admitted = time.perf_counter()
            self.resident += need
            self.peak_resident = max(self.peak_resident, self.resident)
            self.admitted.append(r)

    def _launch(self) -> None:
        for slot in self.ex.idle_slots():
            if slot in self.running or not self.admitted:
                continue
            batch, px = [], 0
            while (self.admitted and len(batch) < self.ex.slot_tiles
                   and px + self.admitted[0].pixels <= self.ex.slot_pixels):
                r = self.admitted.popleft()
                batch.append(r)
                px += r.pixels
            if not batch:
                continue
            try:
                self.ex.launch(slot, batch)
            except Exception as e:  # the batch fails, the server goes on
                now = time.perf_counter()
                for r in batch:
                    r.error, r.done, r.staged = f"launch failed: {e}", now, None
                    self.resident -= self.tile_bytes(r)
                    self.finished.append(r)
                continue
            now = time.perf_counter()
            for r in batch:
                r.started = now
            self.running[slot] = batch
        self.max_inflight = max(self.max_inflight, len(self.running))

    def step(self) -> None:
        self._complete()
        self._admit()
        self._launch()

    def drain(self, idle_sleep: float = 0.0002) -> None:
        while self.busy():
            self.step()
            time.sleep(idle_sleep)

    def run_trace(self, arrivals, images, idle_sleep: float = 0.0002) -> list:
        """Submit images[i] at arrivals[i] seconds after the start, in real
        time, and serve until every request has finished."""
        t0 = time.perf_counter()
        i, n = 0, len(arrivals)
        while i < n or self.busy():
            now = time.perf_counter() - t0
            while i < n and arrivals[i] <= now:
                self.submit(Request(i, images[i], t0 + arrivals[i]))
                i += 1
            self.step()
            time.sleep(idle_sleep)
        return sorted(self.finished + self.rejected, key=lambda r: r.rid)


class _GpuSlots:
    """What both GPU executors share: per-slot streams, staging of host
    tiles on a copy stream (tiles already on the device are used in place),
    start/end events around each slot's work and the read-back of results."""

    def _init_slots(self, plan, n_slots: int, keep_blobs: bool):
        import torch
        self.torch = torch
        self.plan = plan
        self.bytes_per_pixel = 1 if plan.dtype == "u8" else 4
        self.keep_blobs = keep_blobs
        self.copy_stream = torch.cuda.Stream()
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.events = [None] * n_slots
        self.starts = [None] * n_slots
        self.batches = [None] * n_slots

    def stage(self, r: Request):
        torch = self.torch
        if getattr(r.image, "is_cuda", False):
            return r.image, None
        with torch.cuda.stream(self.copy_stream):
            dev = torch.empty(r.image.shape, dtype=r.image.dtype, device=self.plan.device)
            dev.copy_(r.image, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        return dev, ev

    def idle_slots(self):
        return [i for i, b in enumerate(self.batches) if b is None]

    def _begin(self, slot: int, batch):
        s = self.streams[slot]
        for r in batch:
            dev, ev = r.staged
            if ev is not None:
                s.wait_event(ev)
                dev.record_stream(s)
        start = self.torch.cuda.Event(enable_timing=True)
        start.record(s)
        self.starts[slot] = start
        return s

    def _end(self, slot: int, batch):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.streams[slot])
        self.events[slot] = ev
        self.batches[slot] = batch

    def _results(self, slot: int, n: int):
        """(result words [n, 4], blob records or None) of the slot's batch."""
        raise NotImplementedError

    def poll(self, slot: int):
        """None while the slot's batch runs; then one (count, n_candidates,
        flags, density, blobs, device ms) tuple per tile, or the exception
        that the read-back raised for every tile of the batch."""
        ev = self.events[slot]
        try:
            if ev is None or not ev.query():
                return None
            n = len(self.batches[slot])
            with self.torch.cuda.stream(self.streams[slot]):
                res, blobs = self._results(slot, n)
            dev_ms = self.starts[slot].elapsed_time(ev)
        except Exception as e:
            n = len(self.batches[slot]) if self.batches[slot] else 0
            self.events[slot] = None
            self.batches[slot] = None
            return [e] * n
        dens = res[:, 3].copy().view(np.float64)
        out = []
        for i in range(n):
            cnt = int(res[i, 0])
            b = blobs[i][: min(cnt, len(blobs[i]))].copy() if blobs is not None else None
            out.append((cnt, int(res[i, 1]), int(res[i, 2]) & 0xFFFFFFFF, float(dens[i]), b,
                        dev_ms))
        self.events[slot] = None
        self.batches[slot] = None
        return out


class GpuExecutor(_GpuSlots):
    """Slots = BatchRunners (mhfd_detect_batched), each with its own stream;
    tile copies on a separate copy stream."""

    def __init__(self, plan, n_slots: int = 2, slot_tiles: int = 32, slot_pixels: int = 1 << 27,
                 capacity: int = 1 << 16, autotuner=None, keep_blobs: bool = False,
                 lanes: int = 1):
        from .batch import BatchRunner
        self._init_slots(plan, n_slots, keep_blobs)
        self.slot_tiles, self.slot_pixels = slot_tiles, slot_pixels
        self.autotuner = autotuner
        self.runners = [BatchRunner(plan, slot_tiles, slot_pixels, capacity, lanes)
                        for _ in range(n_slots)]
        self.fixed_bytes = sum(r.ws_bytes + r.blobs.numel() * 4 + r.results.numel() * 8
                               for r in self.runners)

    def launch(self, slot: int, batch) -> None:
        s = self._begin(slot, batch)
        imgs = [r.staged[0] for r in batch]
        segs = ([self.autotuner.seg_rows_for(r.h, r.w) for r in batch]
                if self.autotuner else None)
        runner = self.runners[slot]
        runner.set_tiles(imgs, segs, stream=s)
        runner.run(s)
        self._end(slot, batch)

    def _results(self, slot: int, n: int):
        runner = self.runners[slot]
        res = runner.results[:n].cpu().numpy()
        blobs = runner.blobs[:n].cpu().numpy() if self.keep_blobs else None
        return res, blobs


class PlainExecutor(_GpuSlots):
    """The comparison point of the batched server: the same scheduler, but
    every slot runs one tile at a time through plain mhfd_detect calls on its
    own stream (no batching), with workspaces for the largest tile."""

    def __init__(self, plan, n_slots: int = 3, max_h: int = 8192, max_w: int = 8192,
                 capacity: int = 1 << 16, keep_blobs: bool = False):
        import torch
        self._init_slots(plan, n_slots, keep_blobs)
        self.slot_tiles, self.slot_pixels = 1, max_h * max_w
        nb = plan.detect_workspace_bytes(max_h, max_w)
        dev = plan.device
        self.ws = [torch.empty(nb, dtype=torch.uint8, device=dev) for _ in range(n_slots)]
        self.raw = [torch.empty((capacity, 5), dtype=torch.int32, device=dev)
                    for _ in range(n_slots)]
        self.res = [torch.zeros((1, 4), dtype=torch.int64, device=dev) for _ in range(n_slots)]
        self.capacity = capacity
        self.fixed_bytes = n_slots * (nb + capacity * 20 + 32)

    def launch(self, slot: int, batch) -> None:
        s = self._begin(slot, batch)
        (r,) = batch
        self.plan.detect_into(r.staged[0], self.raw[slot], self.res[slot][0], None,
                              self.ws[slot], stream=s)
        self._end(slot, batch)

    def _results(self, slot: int, n: int):
        res = self.res[slot][:n].cpu().numpy()
        blobs = self.raw[slot][None].cpu().numpy() if self.keep_blobs else None
        return res, blobs


def summarize(reqs, wall: float) -> dict:
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    dev = np.array([r.device_ms for r in ok if r.device_ms >= 0])
    mpix = sum(r.pixels for r in ok) / 1e6
    pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None  # noqa: E731
    return {"requests": len(reqs), "served": len(ok),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "device_p50_ms": pct(dev, 50), "device_p99_ms": pct(dev, 99),
            "mpix": mpix, "mpix_per_s": mpix / wall}
