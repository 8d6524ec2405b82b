"""Autotuner for the batched path (glint_shade_batched).

Times every candidate launch shape on the actual views with HIP events and
returns the fastest: tile shape (tile_w x tile_h = 64 pixels per wave) and
persistent workgroups per compute unit, or one workgroup per tile.  Outputs
do not depend on the shape (each pixel's arithmetic and summation order are
fixed), so tuning never changes the image.
"""
from __future__ import annotations

import itertools

import torch

from . import glint

TILES = ((8, 8), (16, 4), (32, 2), (64, 1))
BLOCKS_PER_CU = (0, 4, 8, 16, 32)      # 0: one workgroup per tile instead of persistent workgroups


def autotune(gbufs, outs, materials, lights, tiles=TILES, blocks_per_cu=BLOCKS_PER_CU, reps=2,
             k_max=4, n_probe_max=21, rounding=0, use_graph=False):
    """Returns ((tile_w, tile_h, blocks_per_cu), {shape: ms})."""
    stream = torch.cuda.current_stream()
    timings = {}
    for (tw, th), bpc in itertools.product(tiles, blocks_per_cu):
        plan = glint.GlintPlan(gbufs, outs, materials, lights, k_max=k_max, n_probe_max=n_probe_max,
                               rounding=rounding, tune=(tw, th, bpc))
        plan.run(use_graph=use_graph)               # warm-up (and graph capture)
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            plan.run(use_graph=use_graph)
        e.record(stream)
        torch.cuda.synchronize()
        timings[(tw, th, bpc)] = s.elapsed_time(e) / reps
        plan.close()
    best = min(timings, key=timings.get)
    return best, timings
