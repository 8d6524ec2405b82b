"""Algorithmic work of one glint-shading launch, in VALU issue slots.

The path is ALU-bound (60 bytes of G-buffer and output per pixel against
thousands of VALU operations), so its roofline is the VALU issue rate:
256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane-slots/s.  A slot is
one lane-instruction issue; quarter-rate instructions (32-bit integer
multiply, FP32/FP64 transcendentals and square roots) count 4.

Per-unit costs are the minimal instruction sequences of each step of the
method on gfx950 (the compiler already fuses xor+add into v_xad_u32 and
x ^ (x >> 16) into one SDWA xor):

  hash step H(h, w) = fmix32((h ^ w) + c): xad, xor-shift, mul_lo, shift, xor,
      mul_lo, xor-shift = 5 + 2 x 4 = 13 slots
  live gate (gate probability reaches the smallest uniform 2^-24; the others
      cannot open and need no work): H + compare + mask insert = 15
  open gate (extra): slot-1 angular key (pack 3 + H 13), H 13, inverse normal
      CDF 22, node mean/sigma 9, count 3, bilinear weight and accumulate 5 = 68
  item-light (one pixel, probe, light): FP64 half vector 27, cosines 11, GGX
      ratio 10, angular cell 20, log(1-p) 12, 4 gate set-ups 4 x 19 = 76,
      4 slot-0 angular keys 64, Fresnel 4, Smith masking 16, radiance 3 = 243
  item (one pixel, probe): probe centre 12, 4 x (simplex locate 28 + node hash
      13 + 6 texel-key hashes 78 + 6 LDS stores) = 500, frame 10, FP64
      normalisation of n and w 30 = 552
  pixel: FP64 footprint moments/eigenvalue 60, atan2 60, sincos 60, probe split
      and area level 25, log2 40, cell and tetrahedron 70, weights and record 65 = 380

Units are counted exactly by the library's instrumented kernel (debug
planes).  Loop control, address arithmetic, LDS traffic, recomputation and
idle lanes are not credited, so the achieved rate is a lower bound on the
issue rate the kernel sustains.
"""
from __future__ import annotations

VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9          # lane-slots / s
FP32_PEAK_FLOPS = 157.3e12                       # vendor dense FP32 vector (packed FMA)

HASH = 13
COST = {
    "live_gate": HASH + 2,
    "open_gate": 3 + HASH + HASH + 22 + 9 + 3 + 5,
    "item_light": 27 + 11 + 10 + 20 + 12 + 4 * 19 + 4 * (3 + HASH) + 4 + 16 + 3,
    "item": 12 + 4 * (28 + HASH + 6 * HASH + 6) + 10 + 30,
    "pixel": 380,
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
