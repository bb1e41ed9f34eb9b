"""Autotuner for the launch schedule of the compositing stage.

The wave schedule of `gs_composite` (how many persistent four-wave groups
each compute unit runs, i.e. how the (view, tile, quadrant) work items are
spread and how much gather latency other waves hide, or whether each
quadrant's list is walked by a producer / consumer pair of waves) has no
single best value: few long lists favour pairs or many resident waves, many
short lists favour fewer, dynamically balanced ones.  `tune_composite` times each candidate on the
caller's workload with HIP events on the launch stream (the projected and
binned frame is reused, so only compositing is timed) and leaves the fastest
one set.  Results are cached per shape class in memory (and optionally in a
JSON file).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B

CANDIDATES = (2, 3, 4, 5, 6, 8, "pairs")
_cache: dict = {}


def shape_class(n_views, width, height, n_keys):
    """Workloads that share a best schedule: views, resolution, keys per view (log2 bucket)."""
    per_view = max(1, int(n_keys) // max(1, int(n_views)))
    return "v%d_%dx%d_k2^%d" % (n_views, width, height, int(math.log2(per_view)))


def _apply(c, with_pairs):
    """Set candidate c: a number of four-wave groups per CU (one wave per
    quadrant when pairs are among the candidates, else the current pair
    setting), or "pairs"."""
    if c == "pairs":
        B.set_tuning(composite_pairs=2)
    elif with_pairs:
        B.set_tuning(int(c), composite_pairs=1)
    else:
        B.set_tuning(int(c))


def tune_composite(renderer, frame, n_views, candidates=CANDIDATES, reps=10, cache_path=None):
    """Time gs_composite on `frame` (already projected and binned) for every
    candidate (groups per CU, or "pairs") and keep the fastest.  Returns
    (best, {candidate: ms})."""
    with_pairs = "pairs" in candidates
    n_keys = int(frame.num.item())
    key = shape_class(n_views, renderer.W, renderer.H, n_keys)
    if key in _cache:
        _apply(_cache[key], with_pairs)
        return _cache[key], {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk:
            v = disk[key]
            _cache[key] = v if v == "pairs" else int(v)
            _apply(_cache[key], with_pairs)
            return _cache[key], {}
    times = {}
    for c in candidates:
        _apply(c, with_pairs)
        for _ in range(2):
            renderer.composite(frame, n_views)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            renderer.composite(frame, n_views)
        b.record()
        torch.cuda.synchronize()
        times[c] = a.elapsed_time(b) / reps
    best = min(times, key=times.get)
    _apply(best, with_pairs)
    _cache[key] = best
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = best
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1, sort_keys=True)
    return best, times
