"""Launch-shape autotuner for the batched field kernels.

Times every candidate (block shape x persistent grid size) on a throw-away copy of the
batch, keeps the fastest, and caches the choice in a JSON file keyed by the device
name, precision, dimension and the batch's total node count (bucketed by powers of 2).
"""
from __future__ import annotations

import json
import math
import os

BLOCK_X = (32, 64, 128, 256)
BLOCKS_PER_CU = (2, 4, 8, 16)


def _key(cfgs, device_name):
    nodes = sum(math.prod(c.nodes()) for c in cfgs)
    c0 = cfgs[0]
    return "%s|fp%d|%dd|nodes~2^%d" % (device_name, c0.precision, c0.dim, int(round(math.log2(max(nodes, 1)))))


def tune_batch(cfgs, cache_path=None, steps=6, reps=2, n_cu=None, verbose=False):
    """Returns (block_x, grid_blocks) for a batch of these run configurations."""
    import torch
    from . import binding as B
    dev = torch.cuda.get_device_properties(0)
    n_cu = n_cu or dev.multi_processor_count
    key = _key(cfgs, dev.name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return tuple(cache[key]["launch"])
    probe = B.PmlPicBatch(cfgs, particles_per_run=1, use_graph=True)
    results = []
    for bx in BLOCK_X:
        for bpc in BLOCKS_PER_CU:
            probe.set_launch(bx, bpc * n_cu)
            probe.step(2)
            t = min(probe.timed_steps(steps) for _ in range(reps)) / steps
            results.append((t, bx, bpc * n_cu))
            if verbose:
                print("autotune block_x=%d grid=%d: %.1f us/step" % (bx, bpc * n_cu, t * 1e6), flush=True)
    probe.close()
    del probe
    t, bx, grid = min(results)
    if cache_path:
        cache[key] = {"launch": [bx, grid], "us_per_step": t * 1e6,
                      "candidates": [[r[1], r[2], r[0] * 1e6] for r in results]}
        d = os.path.dirname(cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return bx, grid
