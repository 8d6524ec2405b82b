"""Algorithmic work of one glint-shading launch, in VALU issue slots.

The path is ALU-bound (60 bytes of G-buffer and output per pixel against
thousands of VALU operations), so its roofline is the FP32 VALU issue rate.

Peak.  A gfx950 SIMD issues 64-lane FP32/INT32 VALU instructions at one per
two clocks when at least two waves are resident (one wave alone issues one
per four clocks), i.e. 32 lane-operations per clock per SIMD:
    256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.64e12 lane-slots/s,
the vendor's FP32 vector peak (157.3 TFLOP/s) counted as FMAs.  valu_probe
(built with the library) measures 0.42-0.47 wave-instructions per clock per
SIMD for v_mul_f32 at 16 waves per SIMD and 0.21 with one wave.

Slot costs.  One slot is one lane-operation at that rate; the probe's rates
per instruction class give
    FP32 add/mul/FMA/compare/select, INT32 add/logic/shift, cvt  1
    v_mul_lo_u32, FP64 add/mul/FMA/compare/convert                2
    FP32 exp/log/rcp/rsq/sqrt                                     4
    FP64 rcp/rsq seeds                                            8
FP64 1/sqrt(x) and 1/x, which need only be accurate to about 1e-14 on this
path, are a seed (within 6e-8 on gfx950) and one Newton step: 8 + 4 FP64
operations = 16 slots, 8 + 2 = 12 slots; a correctly rounded FP64 quotient
or square root (kept where a decision can sit exactly on its boundary) is
counted as 20 and 24.

Per-unit costs: the minimal instruction sequence of each step of the method
at the path's precision (FP64 for the footprint, the grid transforms, the
half vector and the angular projection; FP32 for the rest; exact integers for
keys and gates):

  hash step H(h, w) = fmix32((h ^ w) + c): xor-add, xor-shift, mul_lo, shift,
      xor, mul_lo, xor-shift = 5 + 2 x 2 = 9
  live gate (its node's gate probability reaches the smallest uniform 2^-24;
      the others provably cannot open and need no work): the hash head (H
      without fmix32's last xor-shift, which keeps the top 16 bits, so
      H <= t implies head <= t | 0xFFFF, and for t below 2^16 the head
      decides the gate exactly) 8, then a share of the node's test whether
      any of its twelve gates can have opened (five three-input minimums
      and one compare per twelve gates, 0.5, rounded up to 1) = 9, with
      thresholds below 2^16 (live_gate_small) or not.  Gates open rarely,
      so which of a node's gates opened is worked out only for an open gate
      (below).
  open gate (extra): locating it among its node's twelve words (the
      twelve hashes' last steps and 12 compares) 24, slot-1 angular key
      (pack 3 + H) 12, H 9, inverse normal CDF (bits to x, 1-x, 1+x 7,
      log 6, select 1, polynomial 9, scale 2) 25, node mean/sigma 11,
      Gaussian 1, count 2, bilinear weight and accumulate 5 = 89
  pixel-light (one pixel and one light: everything here depends on the
      pixel and the light only, never on the probe, so it is credited once
      per valid (pixel, light) pair however many probes the pixel has; the
      unit half vector enters through dot products: |wi + wo|^2 = 2 (1 +
      <wi,wo>) and so on): <n,wo> and its sign 8, <wi,wo> 6, |wi + wo|^2 and
      guard 4, 1/|wi + wo| 16, <n,h> 4, cos^2/sin^2 8, GGX ratio p 12,
      angular coordinates, cell and bilinear fractions 46 (the frame
      projections <t,wo>, <b,wo>: 4 FP64 operations), log(1-p) 21, 4 gate
      set-ups (the node's trials are per pixel: trials x log, 1-exp, guards,
      threshold, shift) 4 x 28 = 112, 4 slot-0 angular keys 4 x 12 = 48 = 285
  lit pixel-light (extra, when at least one gate of the light opened in
      some probe of the pixel; otherwise the light adds exactly nothing):
      Fresnel 13, Smith Lambda(wo) 20, radiance factor and RGB 13 = 46
  item (one pixel, probe, for the pixels where some gate of some light can
      open: the others shade to exactly 0 and need no probe work; only what
      depends on the probe's centre): probe
      centre 28, 4 x (key unpack 5, trig table index 3, rotation 8,
      anisotropic scales 14, lattice shear/floor/fractions 18, triangle 2,
      vertex selects 6, barycentrics 10, texel keys H(H(node, i), j) of the
      three vertices, which span two lattice columns: 2 + 3 hashes 45 and the
      column select 2) = 4 x 113 = 452, probe sum 3 = 483
  pixel: density 5, FP64 normalisation of n and w 68, footprint moments 24,
      <n,wi> 6, eigenvalue and ratio 60, atan2 80, sigma0 times the major-axis
      eigenvector 58, probe split 50, area level 6, ratio/orientation cell,
      triangle, merge, sort, tetrahedron and node words 180,
      D(n)/(R N P 4<wi,n>) and Lambda(wi) 56, FP64 tangent frame of n in
      implicit form (sign s, a = -1/(s + n_z), s n_x) 17, <n,wi> and <wi,t>,
      <wi,b> from it 14, the 4 nodes' base hashes H(material, node) 36 = 660

Adjoint (glint_shade_backward with the forward's lit masks): the minimal
work to differentiate the relaxed forward is, per lit pixel (a light opened a
gate in it) its set-up (pixel, above); per lit probe its texel keys (item);
per lit (pixel, light) the light's set-up (pixel-light) and the gradient
algebra below; per (probe, light) pair with an open gate its live gates
again (to find the open ones: hash, compare and bit, 12 each); per open gate
the forward's count (without the forward's locating steps and compares) and the
derivative terms below.
  lit pixel-light gradient algebra: Fresnel and Lambda(wo) 33, cos^2/sin^2
      6, dp/dalpha and dp/d<n,h>^2 12, dLambda(wo)/d(c, alpha) 14, G 7,
      dG/dalpha 10, the alpha and ln N sums 13, the unit half vector (FP64)
      6, 1 - <wi,h> 6, the Fresnel, normal and frame terms 17, the frame
      axes (FP64) 24, gradient w.r.t. h 21, the Lambda(wo) term 6, the chain
      through h = (wi + wo)/|wi + wo| and wo = d/|d| 31 = 206
  open gate derivative terms (extra): 1/(2 sigma) 6, dsigma/dp and
      dsigma/dm 7, dm/d ln N 2, the five accumulations with their weights
      15 = 30

Units are counted exactly by the library's instrumented kernel (debug
planes): pixel-lights from the gated binomials each light evaluates per
probe, lit pixel-lights from the per-light count sums.  Loop control,
address arithmetic, LDS traffic, recomputation (a pixel's light set-up or its
node hashes done again for each of its probes), scheduling and idle lanes are
not credited, so the achieved rate is a lower bound on the issue rate the
kernel sustains.
"""
from __future__ import annotations

CU, SIMD_PER_CU, LANES_PER_CLK, CLOCK_HZ = 256, 4, 32, 2.4e9
VALU_PEAK_SLOTS = CU * SIMD_PER_CU * LANES_PER_CLK * CLOCK_HZ    # lane-slots / s (78.64e12)
FP32_PEAK_FLOPS = 157.3e12                                       # vendor dense FP32 vector (FMA = 2 flops)

HASH = 5 + 2 * 2
FP64_RSQ = 8 + 4 * 2
FP64_RCP = 8 + 2 * 2
FP64_DIV, FP64_SQRT = 20, 24
COST = {
    "live_gate": HASH - 1 + 1,
    "live_gate_small": HASH - 1 + 1,
    "open_gate": 12 + 12 + (3 + HASH) + HASH + 25 + 11 + 1 + 2 + 5,
    "pixel_light": 8 + 6 + 4 + FP64_RSQ + 4 + 8 + 12 + 46 + 21 + 4 * 28 + 4 * (3 + HASH),
    "pixel_light_lit": 13 + 20 + 13,
    "item": (8 + FP64_RCP + 8) + 4 * (5 + 3 + 8 + 14 + 18 + 2 + 6 + 10 + 5 * HASH + 2) + 3,
    "pixel": (5 + 2 * (12 + FP64_RSQ + 6) + 24 + 6 + (12 + FP64_SQRT + 2 + FP64_DIV + 2) + 80
              + (26 + 2 * FP64_RSQ) + (8 + 2 * FP64_DIV + 2) + 6 + 180 + 56
              + (5 + FP64_RCP) + 6 + 8 + 4 * HASH),
}


BWD_COST = {
    "pixel": COST["pixel"],
    "item": COST["item"],
    "pixel_light": COST["pixel_light"] + 206,
    # nearly every gate block of the adjoint holds an open gate: each gate is
    # hashed, compared and its bit inserted (H + 3), and the open gates are
    # then located from the bits (no extra compares)
    "live_gate": HASH + 1 + 2,
    "open_gate": (COST["open_gate"] - 24) + 30,
}


def units_from_debug(dbg):
    """Unit counts from the debug planes of one launch (numpy arrays).

    Every probe of a pixel evaluates the same lights, each with 12 gated
    binomials per grid node, so a pixel's valid lights number
    n_gate / (12 n_nodes n_probe); a light is lit in a pixel when its count
    sum b (b_light) is positive, which needs an open gate."""
    import numpy as np
    flags = dbg["flags"].astype(np.int64) & 0xFFFFFFFF
    shaded = (flags & 1) > 0
    n_nodes = (dbg["cell"].astype(np.int64) >> 15) & 7
    n_probe = dbg["n_probe"].astype(np.int64)
    n_gate = dbg["n_gate"].astype(np.int64) & 0xFFFFFFFF
    ok = shaded & (n_nodes > 0)
    item_lights = np.where(ok, n_gate // np.maximum(12 * n_nodes, 1), 0)
    pixel_lights = np.where(ok, n_gate // np.maximum(12 * n_nodes * n_probe, 1), 0)
    live = int((dbg["n_live"].astype(np.int64) & 0xFFFFFFFF).sum())
    small = int((dbg["n_live_small"].astype(np.int64) & 0xFFFFFFFF).sum()) if "n_live_small" in dbg else 0
    lit_pl = int(((dbg["b_light"] > 0) & shaded[None]).sum()) if "b_light" in dbg else 0
    # items only of pixels where some gate can open: the others shade to
    # exactly 0 and need no item (their light set-up decides it)
    n_live = dbg["n_live"].astype(np.int64) & 0xFFFFFFFF
    return {
        "pixel": int(shaded.sum()),
        "item": int(n_probe[shaded & (n_live > 0)].sum()),
        "pixel_light": int(pixel_lights.sum()),
        "pixel_light_lit": lit_pl,
        "live_gate": live - small,
        "live_gate_small": small,
        "open_gate": int((dbg["n_open"].astype(np.int64) & 0xFFFFFFFF).sum()),
        # not priced (reported for the record): item-lights and all gates
        "item_light": int(item_lights.sum()),
        "item_light_lit": int((dbg["n_lit"].astype(np.int64) & 0xFFFFFFFF).sum()) if "n_lit" in dbg else 0,
        "gate": int(n_gate.sum()),
    }


def bwd_units(dbg, lit, probes):
    """Units of the adjoint from the instrumented forward's planes and the
    lit masks of glint_shade_lit (numpy arrays): lit pixels, lit probes
    (set bits of the probe mask; bit 31 stands for probes 31 on, so it is
    expanded from the pixel's probe count), lit (pixel, light) pairs, the live
    gates of the (probe, light) pairs with an open gate, open gates."""
    import numpy as np
    lit = lit.astype(np.int64) & 0xFFFF
    pm = probes.astype(np.int64) & 0xFFFFFFFF
    npr = dbg["n_probe"].astype(np.int64)
    low = np.unpackbits((pm & 0x7FFFFFFF).astype("<u4").view(np.uint8)).reshape(pm.shape + (32,)).sum(-1)
    hi = np.where((pm >> 31) & 1, np.maximum(npr - 31, 1), 0)
    return {
        "pixel": int((lit != 0).sum()),
        "item": int((low + hi).sum()),
        "pixel_light": int(np.unpackbits(lit.astype("<u2").view(np.uint8)).sum()),
        "live_gate": int((dbg["n_live_lit"].astype(np.int64) & 0xFFFFFFFF).sum()),
        "open_gate": int((dbg["n_open"].astype(np.int64) & 0xFFFFFFFF).sum()),
    }


def slots(units, cost=None):
    cost = COST if cost is None else cost
    return sum(cost[k] * units[k] for k in cost)
