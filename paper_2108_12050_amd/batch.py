"""Batched detection of tiles of different sizes (mhfd_detect_batched).

``BatchRunner`` owns everything the batched call touches -- the device table
of tile descriptors, the workspace and the per-tile outputs -- at fixed
addresses, so one HIP graph captured around ``run()`` can be replayed after
``set_tiles()`` has written new descriptors (new images, other sizes within
the bounds) without capturing again.
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
    most ``max_pixels`` pixels, each with room for ``capacity`` blobs."""

    def __init__(self, plan: Plan, max_tiles: int, max_pixels: int, capacity: int):
        self.plan = plan
        self.L = plan._L
        self.max_tiles, self.max_pixels, self.capacity = int(max_tiles), int(max_pixels), int(capacity)
        dev = plan.device
        self.ws_bytes = int(self.L.mhfd_batch_workspace_size(plan._handle, self.max_tiles,
                                                             self.max_pixels))
        if self.ws_bytes == 0:
            raise _lib.MHFDError(1, "mhfd_batch_workspace_size",
                                 f"{max_tiles} tiles / {max_pixels} pixels out of range")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.table = torch.zeros(self.max_tiles * TILE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self.blobs = torch.empty((self.max_tiles, self.capacity, 5), dtype=torch.int32, device=dev)
        self.results = torch.zeros((self.max_tiles, _lib.RESULT_WORDS), dtype=torch.int64,
                                   device=dev)
        self.n = 0
        self._imgs = []

    def set_tiles(self, imgs, seg_rows=None, stream=None) -> None:
        """Write descriptors for `imgs` (device tensors of the plan's dtype,
        rows contiguous) into the device table, on `stream` (default: the
        current stream).  The tensors must stay alive while the batch runs."""
        n = len(imgs)
        if not 1 <= n <= self.max_tiles:
            raise ValueError(f"{n} tiles, runner holds 1..{self.max_tiles}")
        want = torch.uint8 if self.plan.dtype == "u8" else torch.float32
        t = np.zeros(n, dtype=TILE_DTYPE)
        for i, im in enumerate(imgs):
            if im.dim() != 2 or im.dtype != want or im.device != self.plan.device or im.stride(1) != 1:
                raise ValueError(f"tile {i}: expected a 2-D {want} tensor with contiguous rows "
                                 f"on {self.plan.device}")
            t[i]["img"] = im.data_ptr()
            t[i]["h"], t[i]["w"] = im.shape
            t[i]["pitch"] = im.stride(0)
            t[i]["blobs"] = self.blobs[i].data_ptr()
            t[i]["result"] = self.results[i].data_ptr()
            t[i]["capacity"] = self.capacity
            t[i]["seg_rows"] = 0 if seg_rows is None else int(seg_rows[i])
        host = torch.from_numpy(t.view(np.uint8).copy())
        s = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            self.table[: host.numel()].copy_(host.pin_memory(), non_blocking=True)
        self._keep = host
        self.n = n
        self._imgs = list(imgs)

    def run(self, stream=None) -> None:
        """Enqueue mhfd_detect_batched for the current table (no sync)."""
        st = self.L.mhfd_detect_batched(self.plan._handle, self.n, self.table.data_ptr(),
                                        self.max_pixels, self.ws.data_ptr(), self.ws_bytes,
                                        _stream_ptr(stream))
        _lib.check(st, "mhfd_detect_batched")

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


def detect_batched(plan: Plan, imgs, capacity: int = 1 << 16, seg_rows=None) -> list:
    """One-shot batched detection of a list of device images."""
    px = sum(int(i.shape[0]) * int(i.shape[1]) for i in imgs)
    r = BatchRunner(plan, len(imgs), px, capacity)
    r.set_tiles(imgs, seg_rows)
    r.run()
    return r.detections()
