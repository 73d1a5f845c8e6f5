"""Autotuner for the batched detector's per-size-class launch parameter.

The LoG strip kernel gives each workgroup one (scale, 64-column strip,
segment of rows).  The strip width and the 32-row chunk are fixed by the
register and LDS layout, and a workgroup holds one scale.  What remains free
is the segment height: every segment recomputes a 2R-row halo of row-pass
results before its first output row, so tall segments waste less work,
while short segments give more workgroups to balance across the 256 compute
units.  The best height depends on the tile size and the plan's radii.

`Autotuner.tune` times mhfd_detect_batched on a synthetic tile of each size
class for each candidate height (HIP events, median of repeats), keeps the
fastest, and caches the choice in a JSON file keyed by GPU architecture,
library build and plan (scales, radii, dtype).  `seg_rows_for` returns the
tuned height for a tile (nearest size class by pixel count), or 0 -- the
library default -- when nothing was tuned.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import _lib
from .api import Plan
from .batch import BatchRunner

CANDIDATES = (64, 128, 256, 384, 512, 768, 1024)


def _lib_hash() -> str:
    with open(_lib.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


class Autotuner:
    def __init__(self, plan: Plan, cache_path: str | None = None):
        self.plan = plan
        self.cache_path = cache_path
        self.table: dict[tuple[int, int], int] = {}
        self.key = json.dumps({"arch": _arch(), "lib": _lib_hash(), "sigmas": plan.sigmas,
                               "radii": plan.radii, "dtype": plan.dtype}, sort_keys=True)
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                entry = json.load(f).get(self.key)
            if entry:
                self.table = {tuple(map(int, k.split("x"))): int(v) for k, v in entry.items()}

    def _tile(self, h: int, w: int, seed: int) -> torch.Tensor:
        from . import synth
        if self.plan.dtype == "u8":
            a = synth.sem_tile(seed, 0.0, h, w)
        else:
            a = synth.blob_field(seed, h, w)
        return torch.from_numpy(a).to(self.plan.device)

    def time_one(self, tile: torch.Tensor, seg: int, reps: int = 5) -> float:
        """Median device milliseconds of one batched detection of `tile`."""
        r = BatchRunner(self.plan, 1, tile.numel(), 1 << 12)
        r.set_tiles([tile], seg_rows=[seg])
        r.run()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            r.run()
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.median(times))

    def tune(self, sizes, candidates=CANDIDATES, reps: int = 5) -> dict:
        """Tune each (h, w) in `sizes`; returns {size: (best_seg, {seg: ms})}."""
        report = {}
        for i, (h, w) in enumerate(sizes):
            tile = self._tile(int(h), int(w), 500 + i)
            cands = [c for c in candidates if c <= max(32, (h + 31) // 32 * 32)] or [32]
            t = {c: self.time_one(tile, c, reps) for c in cands}
            best = min(t, key=t.get)
            self.table[(int(h), int(w))] = best
            report[(int(h), int(w))] = (best, t)
        if self.cache_path:
            data = {}
            if os.path.exists(self.cache_path):
                with open(self.cache_path) as f:
                    data = json.load(f)
            data[self.key] = {f"{h}x{w}": s for (h, w), s in self.table.items()}
            with open(self.cache_path, "w") as f:
                json.dump(data, f, indent=1)
        return report

    def seg_rows_for(self, h: int, w: int) -> int:
        if not self.table:
            return 0
        if (h, w) in self.table:
            return self.table[(h, w)]
        px = h * w
        near = min(self.table, key=lambda s: abs(np.log(s[0] * s[1]) - np.log(px)))
        return self.table[near]
