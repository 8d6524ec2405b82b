"""Algorithmic work of one glint-shading launch, in VALU issue slots.

The path is ALU-bound (about 60 bytes of G-buffer per pixel against
thousands of VALU operations), so its roofline is the VALU issue rate of
the chip:  256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane-slots/s.
A slot is one lane-instruction issue; quarter-rate instructions (32-bit
integer multiply, FP32/FP64 transcendentals, FP64 square root) count 4.

Per-unit costs are the minimal instruction counts of each step of the
method as implemented (hash H(h,w) = xor, add, 3 x (shift, xor), 2 x mul_lo
= 8 instructions, 16 slots).  Units are counted exactly by the library's
instrumented kernel (debug planes):

  live gate    a gated binomial whose gate probability reaches 2^-24
               (the others cannot open and need no work): H + shift + compare
  open gate    extra work of an open gate: second H, inverse normal CDF,
               count and weighted accumulate
  item-light   one (pixel, probe, light): half vector (FP64), NDF ratio, angular
               cell (FP64), 8 angular key hashes, log1p, 4 gate set-ups
               (expm1, threshold, mu, sigma), Fresnel, Smith masking, output
  item         one (pixel, probe): probe centre, 4 grid transforms and simplex
               locates (FP64), 4 node hashes, 12 x 2 texel key hashes
  pixel        footprint (FP64 moments, sqrt, atan2, sincos), probe count,
               area / ratio / orientation cell, tetrahedron, weights (FP64 log2)

Anything the kernel does beyond these counts (recomputation, address
arithmetic, loop control, LDS traffic) is not credited, so the achieved rate
is a lower bound on the useful issue rate.
"""
from __future__ import annotations

VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9          # lane-slots / s
FP32_PEAK_FLOPS = 157.3e12                       # vendor dense FP32 vector (packed FMA)

HASH = 16
COST = {
    "live_gate": HASH + 2,
    "open_gate": HASH + 24 + 5,
    "item_light": 23 + 7 + 11 + 24 + 8 * (HASH + 4) + 12 + 4 * 28 + 27,
    "item": 13 + 4 * (3 + HASH + 28 + 2 * 3 * HASH) + 10,
    "pixel": 330,
}


def units_from_debug(dbg):
    """Unit counts from the debug planes of one launch (numpy arrays)."""
    import numpy as np
    flags = dbg["flags"].astype(np.int64) & 0xFFFFFFFF
    shaded = (flags & 1) > 0
    n_nodes = (dbg["cell"].astype(np.int64) >> 15) & 7
    n_gate = dbg["n_gate"].astype(np.int64) & 0xFFFFFFFF
    pairs = np.where(shaded & (n_nodes > 0), n_gate // np.maximum(12 * n_nodes, 1), 0)
    return {
        "pixel": int(shaded.sum()),
        "item": int(dbg["n_probe"][shaded].astype(np.int64).sum()),
        "item_light": int(pairs.sum()),
        "live_gate": int((dbg["n_live"].astype(np.int64) & 0xFFFFFFFF).sum()),
        "open_gate": int((dbg["n_open"].astype(np.int64) & 0xFFFFFFFF).sum()),
        "gate": int(n_gate.sum()),
    }


def slots(units):
    return sum(COST[k] * units[k] for k in COST)
