"""Batched detection of tiles of different sizes (mhfd_detect_batched).

``BatchRunner`` owns everything the batched call touches -- the device table
of tile descriptors, the workspace and the per-tile outputs -- at fixed
addresses, so one HIP graph captured around ``run()`` can be replayed after
``set_tiles()`` has written new descriptors (new images, other sizes within
the bounds) without capturing again.

With ``lanes`` > 1 the tiles are dealt, largest first, to that many
sub-batches of near-equal pixel counts, each one mhfd_detect_batched call
with its own workspace on its own stream, forked from and joined back to
the caller's stream (and captured the same way): the phases of one
sub-batch (LoG, maxima, the small tail launches) overlap those of the
others, as independent per-tile calls on several streams overlap.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from .api import Detection, Plan, _stream_ptr, result_density, split_blobs

TILE_DTYPE = np.dtype([("img", "<u8"), ("h", "<i4"), ("w", "<i4"), ("pitch", "<i8"),
                       ("blobs", "<u8"), ("result", "<u8"), ("capacity", "<i4"),
                       ("seg_rows", "<i4")])
assert TILE_DTYPE.itemsize == C.sizeof(_lib.Tile)


class BatchRunner:
    """Fixed-address state for batches of up to ``max_tiles`` tiles holding at
    most ``max_pixels`` pixels, each with room for ``capacity`` blobs, run as
    ``lanes`` concurrent sub-batches."""

    def __init__(self, plan: Plan, max_tiles: int, max_pixels: int, capacity: int,
                 lanes: int = 1, log_groups_per_cu: int = 0, nms_groups_per_cu: int = 0):
        self.plan = plan
        self.L = plan._L
        self.max_tiles, self.max_pixels, self.capacity = int(max_tiles), int(max_pixels), int(capacity)
        self.lanes = max(1, min(int(lanes), self.max_tiles))
        dev = plan.device
        # snake dealing of tiles sorted by size keeps every lane within
        # total / lanes + one tile
        self.lane_pixels = (self.max_pixels if self.lanes == 1 else
                            min(self.max_pixels, -(-self.max_pixels // self.lanes)
                                + plan.max_h * plan.max_w))
        self.lane_ws_bytes = int(self.L.mhfd_batch_workspace_size(plan._handle, self.max_tiles,
                                                                  self.lane_pixels))
        if self.lane_ws_bytes == 0:
            raise _lib.MHFDError(1, "mhfd_batch_workspace_size",
                                 f"{max_tiles} tiles / {self.lane_pixels} pixels out of range")
        self.ws_bytes = self.lane_ws_bytes * self.lanes
        self.ws = [torch.empty(self.lane_ws_bytes, dtype=torch.uint8, device=dev)
                   for _ in range(self.lanes)]
        self.table = torch.zeros(self.lanes * self.max_tiles * TILE_DTYPE.itemsize,
                                 dtype=torch.uint8, device=dev)
        self.blobs = torch.empty((self.max_tiles, self.capacity, 5), dtype=torch.int32, device=dev)
        self.results = torch.zeros((self.max_tiles, _lib.RESULT_WORDS), dtype=torch.int64,
                                   device=dev)
        self.streams = [torch.cuda.Stream() for _ in range(self.lanes - 1)]
        # launch shape of every call (0: the library's default)
        self.opts = _lib.BatchOpts(int(log_groups_per_cu), int(nms_groups_per_cu))
        self.n = 0
        self.lane_n = [0] * self.lanes
        self._imgs = []

    def set_tiles(self, imgs, seg_rows=None, stream=None) -> None:
        """Write descriptors for `imgs` (device tensors of the plan's dtype,
        rows contiguous) into the device table, on `stream` (default: the
        current stream).  The tensors must stay alive while the batch runs.
        A graph captured by `capture` processes the tile count it was
        captured with: replay it after set_tiles with that many tiles (with
        one lane, fewer tiles also run, and the later descriptors of the
        capture are processed again as they were)."""
        n = len(imgs)
        if not 1 <= n <= self.max_tiles:
            raise ValueError(f"{n} tiles, runner holds 1..{self.max_tiles}")
        want = torch.uint8 if self.plan.dtype == "u8" else torch.float32
        for i, im in enumerate(imgs):
            if im.dim() != 2 or im.dtype != want or im.device != self.plan.device or im.stride(1) != 1:
                raise ValueError(f"tile {i}: expected a 2-D {want} tensor with contiguous rows "
                                 f"on {self.plan.device}")
        # deal tiles largest first in snake order (lanes 0, 1, .., L-1, L-1,
        # .., 0, 0, ..): near-equal pixels per lane, and tile counts per lane
        # that depend on n only, so a captured graph stays valid for new
        # tiles of any sizes
        lanes = [[] for _ in range(self.lanes)]
        for rank, i in enumerate(sorted(range(n), key=lambda i: (-imgs[i].numel(), i))):
            turn, pos = divmod(rank, self.lanes)
            lanes[pos if turn % 2 == 0 else self.lanes - 1 - pos].append(i)
        t = np.zeros(self.lanes * self.max_tiles, dtype=TILE_DTYPE)
        for j, members in enumerate(lanes):
            for q, i in enumerate(sorted(members)):
                im = imgs[i]
                r = t[j * self.max_tiles + q]
                r["img"] = im.data_ptr()
                r["h"], r["w"] = im.shape
                r["pitch"] = im.stride(0)
                r["blobs"] = self.blobs[i].data_ptr()
                r["result"] = self.results[i].data_ptr()
                r["capacity"] = self.capacity
                r["seg_rows"] = 0 if seg_rows is None else int(seg_rows[i])
        self.lane_n = [len(m) for m in lanes]
        # one lane: only the n descriptors written (a graph captured for more
        # tiles keeps reading its later descriptors as they were)
        host = torch.from_numpy((t[:n] if self.lanes == 1 else t).view(np.uint8).copy())
        s = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            self.table[: host.numel()].copy_(host.pin_memory(), non_blocking=True)
        self._keep = host
        self.n = n
        self._imgs = list(imgs)

    def run(self, stream=None) -> None:
        """Enqueue mhfd_detect_batched for every lane's sub-batch (no sync):
        lane 0 on `stream` (default: the current stream), the others on
        side streams that wait for it and that it waits for."""
        main = stream if stream is not None else torch.cuda.current_stream()
        active = [j for j in range(self.lanes) if self.lane_n[j]]
        side = {j: self.streams[j - 1] for j in active if j > 0}
        for st_ in side.values():
            st_.wait_stream(main)
        for j in active:
            st_ = main if j == 0 else side[j]
            table = self.table.data_ptr() + j * self.max_tiles * TILE_DTYPE.itemsize
            status = self.L.mhfd_detect_batched(self.plan._handle, self.lane_n[j], table,
                                                self.lane_pixels, C.byref(self.opts),
                                                self.ws[j].data_ptr(), self.lane_ws_bytes,
                                                int(st_.cuda_stream))
            _lib.check(status, "mhfd_detect_batched")
        for st_ in side.values():
            main.wait_stream(st_)

    def capture(self) -> torch.cuda.CUDAGraph:
        """Capture run() into a HIP graph for the current tile count."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run(s)            # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            self.run()
        return g

    def detections(self) -> list:
        """Per-tile results of the last run (synchronises)."""
        host = self.results[: self.n].cpu()
        res = host.tolist()
        out = []
        for i, (nb, nc, fl, _) in enumerate(res):
            fl &= 0xFFFFFFFF
            if fl & _lib.MHFD_FLAG_INVALID_TILE:
                raise _lib.MHFDError(1, "mhfd_detect_batched", "a tile descriptor failed the "
                                     "device-side checks or the batch exceeded max_pixels")
            if fl & _lib.MHFD_FLAG_CAND_OVERFLOW:
                raise RuntimeError("candidate capacity overflow in the batch")
            yxk, sig, resp = split_blobs(self.blobs[i], min(nb, self.capacity))
            d = Detection(yxk, sig, resp, nb, nc, fl)
            d._density = result_density(host[i])
            out.append(d)
        return out


def detect_batched(plan: Plan, imgs, capacity: int = 1 << 16, seg_rows=None,
                   lanes: int = 1) -> list:
    """One-shot batched detection of a list of device images."""
    px = sum(int(i.shape[0]) * int(i.shape[1]) for i in imgs)
    r = BatchRunner(plan, len(imgs), px, capacity, lanes)
    r.set_tiles(imgs, seg_rows)
    r.run()
    return r.detections()
