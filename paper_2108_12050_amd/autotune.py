"""Autotuner of the batched detector's launch parameters.

The batched form (mhfd_detect_batched) runs the matrix-core LoG as
persistent workgroups that pull (scale, tile, row segment, four 16-column
wave tiles) items, then a persistent maxima pass.  What is free:

  * per size class, the segment height of a tile's LoG items (a multiple of
    32 rows): every segment re-runs its ring's warm-up, 2 nkc - 1 blocks of
    16 intermediate rows per wave, so tall segments waste less work while
    short ones give more items to balance across the 256 compute units;
  * per batch, the launch shape: persistent LoG workgroups per compute unit
    (1, 2 or 4) and maxima workgroups per compute unit (4, 8 or 16)
    (mhfd_batch_opts), and the number of concurrent sub-batches ("lanes",
    one stream each, whose phases overlap).

Fixed by the kernels and therefore not tuned: the 16-column wave tile and
the 32-row K-block of the MFMA operands, the per-scale halo (the exact
column window, R rows above the block), and the scales a workgroup holds
(one per item: its column taps in LDS, a ring per wave; items are numbered
tile-major, so a tile's scales share its image in the caches).

`Autotuner.tune` times one-tile batches of each size class for each
candidate height (HIP events, median of repeats) beside the library default
(0), keeps the fastest, and caches the choice in a JSON file keyed by GPU
architecture, library build and plan (scales, radii, dtype).
`tune_batch_segments` then times a representative batch under each
segment-height rule (the per-class table, the library default, uniform
heights, whole-tile items) and keeps the fastest: in a batch of many tiles
the parallelism comes from the tiles, so the per-class heights, tuned on one
tile alone, are often too short.  `tune_launch` times the batch over the
launch shapes and lanes.  `seg_rows_for` returns the height the kept rule
gives a tile (per class: the nearest size class by pixel count), or 0 -- the
library default -- when nothing was tuned.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os

import numpy as np
import torch

from . import _lib
from .api import Plan
from .batch import BatchRunner

CANDIDATES = (64, 128, 256, 384, 512, 768, 1024)
LOG_GROUPS = (1, 2, 4)
NMS_GROUPS = (4, 8, 16)
LANES = (1, 2, 3)
DEFAULT_LAUNCH = {"log_groups_per_cu": 2, "nms_groups_per_cu": 8, "lanes": 1}
# segment-height rules for a whole batch: the per-class table, uniform
# heights, whole-tile items (height rounded up to 32 rows)
BATCH_RULES = ("per_class", "default", "uniform_1024", "uniform_2048", "whole_tile")


def _lib_hash() -> str:
    with open(_lib.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _median_ms(fn, reps: int) -> float:
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


class Autotuner:
    def __init__(self, plan: Plan, cache_path: str | None = None):
        self.plan = plan
        self.cache_path = cache_path
        self.table: dict[tuple[int, int], int] = {}
        self.launch = dict(DEFAULT_LAUNCH)
        self.batch_rule = "per_class"
        self.key = json.dumps({"arch": _arch(), "lib": _lib_hash(), "sigmas": plan.sigmas,
                               "radii": plan.radii, "dtype": plan.dtype}, sort_keys=True)
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                entry = json.load(f).get(self.key)
            if entry:
                self.table = {tuple(map(int, k.split("x"))): int(v)
                              for k, v in entry.get("seg_rows", {}).items()}
                self.launch.update(entry.get("launch", {}))
                self.batch_rule = entry.get("batch_rule", self.batch_rule)

    def _tile(self, h: int, w: int, seed: int) -> torch.Tensor:
        from . import synth
        if self.plan.dtype == "u8":
            a = synth.sem_tile(seed, 0.0, h, w)
        else:
            a = synth.blob_field(seed, h, w)
        return torch.from_numpy(a).to(self.plan.device)

    def time_one(self, tile: torch.Tensor, seg: int, reps: int = 5) -> float:
        """Median device milliseconds of one batched detection of `tile`
        (seg = 0: the library's default segment height)."""
        r = BatchRunner(self.plan, 1, tile.numel(), 1 << 12)
        r.set_tiles([tile], seg_rows=[seg])
        r.run()
        return _median_ms(r.run, reps)

    def tune(self, sizes, candidates=CANDIDATES, reps: int = 5) -> dict:
        """Tune each (h, w) in `sizes`; returns {size: (best_seg, {seg: ms})},
        where seg 0 is the library default the gain is measured against."""
        report = {}
        for i, (h, w) in enumerate(sizes):
            tile = self._tile(int(h), int(w), 500 + i)
            cands = [c for c in candidates if c <= max(32, (h + 31) // 32 * 32)] or [32]
            t = {c: self.time_one(tile, c, reps) for c in [0] + cands}
            best = min(cands, key=t.get)
            self.table[(int(h), int(w))] = best
            report[(int(h), int(w))] = (best, t)
        self._save()
        return report

    def tune_batch_segments(self, imgs, reps: int = 3) -> dict:
        """Segment heights for a whole batch: a height tuned on one tile of a
        class trades warm-up work for parallelism that a batch of many tiles
        does not need, so the batch `imgs` is timed (default launch shape)
        with the per-class table, with uniform heights and with whole-tile
        items, and the fastest rule is kept for `seg_rows_for`.  Returns
        {"best": rule, "times": {rule: ms}}."""
        px = sum(t.numel() for t in imgs)
        saved = self.batch_rule
        times = {}
        for rule in BATCH_RULES:
            self.batch_rule = rule
            if rule == "per_class" and not self.table:
                continue
            r = BatchRunner(self.plan, len(imgs), px, 1 << 12)
            r.set_tiles(imgs, [self.seg_rows_for(*t.shape) for t in imgs])
            r.run()
            times[rule] = _median_ms(r.run, reps)
            del r
        self.batch_rule = min(times, key=times.get) if times else saved
        self._save()
        return {"best": self.batch_rule, "times": {k: round(v, 3) for k, v in times.items()}}

    def tune_launch(self, imgs, reps: int = 3) -> dict:
        """Time the batch `imgs` (device tiles, tuned segment heights) for
        every launch shape and lane count; keep the fastest.  Returns
        {"best": shape, "default_ms", "best_ms", "times": {shape: ms}}."""
        px = sum(t.numel() for t in imgs)
        segs = [self.seg_rows_for(*t.shape) for t in imgs]
        times = {}
        for lg, ng, ln in itertools.product(LOG_GROUPS, NMS_GROUPS, LANES):
            r = BatchRunner(self.plan, len(imgs), px, 1 << 12, lanes=ln,
                            log_groups_per_cu=lg, nms_groups_per_cu=ng)
            r.set_tiles(imgs, segs)
            r.run()
            times[(lg, ng, ln)] = _median_ms(r.run, reps)
            del r
        best = min(times, key=times.get)
        self.launch = {"log_groups_per_cu": best[0], "nms_groups_per_cu": best[1],
                       "lanes": best[2]}
        self._save()
        d = (DEFAULT_LAUNCH["log_groups_per_cu"], DEFAULT_LAUNCH["nms_groups_per_cu"],
             DEFAULT_LAUNCH["lanes"])
        return {"best": dict(self.launch), "default_ms": times[d], "best_ms": times[best],
                "times": {f"log{k[0]}_nms{k[1]}_lanes{k[2]}": round(v, 3)
                          for k, v in times.items()}}

    def _save(self) -> None:
        if not self.cache_path:
            return
        data = {}
        if os.path.exists(self.cache_path):
            with open(self.cache_path) as f:
                data = json.load(f)
        data[self.key] = {"seg_rows": {f"{h}x{w}": s for (h, w), s in self.table.items()},
                          "launch": self.launch, "batch_rule": self.batch_rule}
        with open(self.cache_path, "w") as f:
            json.dump(data, f, indent=1)

    def seg_rows_for(self, h: int, w: int) -> int:
        if self.batch_rule == "default":
            return 0
        if self.batch_rule.startswith("uniform_"):
            return min(int(self.batch_rule.split("_")[1]), max(32, (h + 31) // 32 * 32))
        if self.batch_rule == "whole_tile":
            return min(4096, max(32, (h + 31) // 32 * 32))
        if not self.table:
            return 0
        if (h, w) in self.table:
            return self.table[(h, w)]
        px = h * w
        near = min(self.table, key=lambda s: abs(np.log(s[0] * s[1]) - np.log(px)))
        return self.table[near]

    def runner(self, max_tiles: int, max_pixels: int, capacity: int) -> BatchRunner:
        """A BatchRunner with the tuned launch shape and lanes."""
        return BatchRunner(self.plan, max_tiles, max_pixels, capacity, self.launch["lanes"],
                           self.launch["log_groups_per_cu"], self.launch["nms_groups_per_cu"])
