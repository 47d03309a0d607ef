"""Autotuner: picks the batched-submit mode, bin tile size (8x8 or 16x16
lists) and bin depth per scene and view-size class by timing the candidates
on the GPU, with a JSON cache.

The choice only affects speed: every mode, tile size and depth gives
bit-identical images.  A (scene, size class) key is the scene's triangle
count, a hash of a sample of its vertices and the power-of-two class of the
views' mean pixel count.  A choice is (mode, bin_depth), where mode carries
VSR_SUBMIT_BIN_TILE16 for 16x16 bin tiles.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import pipeline, vsr

_T16 = vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16
CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (vsr.VSR_SUBMIT_BINNED, 256), (vsr.VSR_SUBMIT_BINNED, 512), (vsr.VSR_SUBMIT_BINNED, 1024),
    (vsr.VSR_SUBMIT_BINNED, 2048), (_T16, 256), (_T16, 512), (_T16, 1024), (_T16, 2048),
    (vsr.VSR_SUBMIT_FUSED, 1024),
)


def describe(choice: Tuple[int, int]) -> dict:
    """Readable form of a (mode, bin_depth) choice."""
    mode, depth = choice
    if mode & 0xFF == vsr.VSR_SUBMIT_FUSED:
        return {"mode": "fused", "tile": 8, "bin_depth": None}
    return {"mode": "binned", "tile": 16 if mode & vsr.VSR_SUBMIT_BIN_TILE16 else 8, "bin_depth": int(depth)}


def scene_key(scene: pipeline.Scene) -> str:
    n = scene.ntri
    if n == 0:
        return "0"
    idx = torch.linspace(0, n - 1, steps=min(n, 64), device=scene.xyz.device).long()
    sample = scene.xyz[:, idx].float().cpu().numpy().tobytes()
    return f"{n}-{hashlib.sha1(sample).hexdigest()[:12]}"


def size_class(views: Sequence[object]) -> int:
    px = sum(int(v.width) * int(v.height) for v in views) / max(1, len(views))
    return int(round(math.log2(max(1.0, px))))


class Tuner:
    def __init__(self, cache_path: Optional[str] = None, candidates=CANDIDATES, reps: int = 3):
        self.cache_path = cache_path
        self.candidates = tuple(candidates)
        self.reps = reps
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self) -> None:
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def choose(self, scene: pipeline.Scene, views: Sequence[object], fmt: int = vsr.VSR_MAP_F32) -> Tuple[int, int]:
        """(mode, bin_depth) for rendering views like these of this scene."""
        key = f"{scene_key(scene)}/{size_class(views)}/{fmt}"
        if key not in self.cache:
            self.cache[key] = self.measure(scene, views, fmt)
            self._save()
        best = self.cache[key]["best"]
        return int(best[0]), int(best[1])

    def measure(self, scene: pipeline.Scene, views: Sequence[object], fmt: int) -> dict:
        times = {}
        for mode, depth in self.candidates:
            b = pipeline.Batch([(scene, v) for v in views], fmt=fmt, mode=mode, bin_depth=depth)
            b.submit()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.reps):
                b.submit()
            e1.record()
            torch.cuda.synchronize()
            times[f"{mode}:{depth}"] = e0.elapsed_time(e1) / self.reps
            del b
        best = min(times, key=times.get)
        mode, depth = (int(x) for x in best.split(":"))
        return {"best": [mode, depth], "ms": times, "views": len(views)}
