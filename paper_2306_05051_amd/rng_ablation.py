"""Hashed uniforms against a precomputed random-number table (Sec. 6.3).

    python -m paper_2306_05051_amd.rng_ablation [--steps 10] [--rounds 3]

The paper reads the two uniforms of each gated binomial from a small texture
of random numbers precomputed at start-up; this library hashes them from the
texel and angular keys.  glint_shade_rng_table shades with the table instead
(word = table[(texel key ^ angular key) mod 2^b]), read either through the
L1/L2 caches or from a per-tile copy in LDS.  This times, on the 4K frame of
the benchmark (3840x2160, 8 GGX materials, 4 lights) and on the paper's
performance setting (1920x1080 plane at 25 degrees, Beckmann alpha = 1.0, one
light), glint_shade against the table variant over table sizes 2^8 ... 2^24
words, alternating the variants over several rounds (HIP events on the launch
stream, same workspace, tile-order pass included in every variant), and
reports each variant's total frame radiance relative to the hashed uniforms:
a table of few words quantises the uniforms, which biases the rare gates
with small opening probabilities.  Prints one JSON object on stdout and a
table on stderr.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

CACHED_LOG2 = (8, 10, 12, 14, 16, 20, 24)
LDS_LOG2 = (8, 10, 12, 13)
TABLE_SEED = 0x5EED


def _variants(glint):
    v = [("hash", None, None)]
    v += [(f"table 2^{b} cached", b, glint.RNG_CACHED) for b in CACHED_LOG2]
    v += [(f"table 2^{b} LDS", b, glint.RNG_LDS) for b in LDS_LOG2]
    return v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rounds", type=int, default=3)
    args = ap.parse_args()

    import torch
    from . import glint, scenes

    frames = []
    gb, mats, lights = scenes.four_k()
    frames.append(("4K bench frame (8 GGX materials, 4 lights)", gb, mats, lights))
    gb, mats, lights = scenes.paper_setting(1920, 1080, view="plane25", log10_density=5.0)
    frames.append(("1080p plane 25 deg, Beckmann alpha=1.0, 1 light", gb, mats, lights))

    stream = torch.cuda.current_stream()
    tables = {b: glint.glint_rng_table_fill(b, TABLE_SEED) for b in sorted(set(CACHED_LOG2) | set(LDS_LOG2))}
    torch.cuda.synchronize()
    result = {"table_seed": TABLE_SEED, "frames": []}
    for name, gb, mats, lights in frames:
        H, W = gb["u"].shape
        dgb = glint.to_device(gb)
        out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        ws = torch.empty(max(1, glint.glint_shade_workspace_bytes(W, H)), dtype=torch.uint8, device="cuda")

        def call(b, placement):
            if b is None:
                glint.glint_shade(dgb, mats, lights, out=out, workspace=ws)
            else:
                glint.glint_shade_rng_table(dgb, mats, lights, tables[b], b, placement, out=out, workspace=ws)

        times = {v[0]: [] for v in _variants(glint)}
        energy = {}
        for rnd in range(args.rounds):
            for label, b, placement in _variants(glint):
                for _ in range(args.warmup):
                    call(b, placement)
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                for _ in range(args.steps):
                    call(b, placement)
                s1.record(stream)
                torch.cuda.synchronize()
                times[label].append(s0.elapsed_time(s1) / args.steps)
                if rnd == 0:
                    energy[label] = float(out.double().sum())
            print(f"{name}: round {rnd + 1} of {args.rounds} done", file=sys.stderr, flush=True)
        rows = []
        base = float(np.median(times["hash"]))
        for label, b, placement in _variants(glint):
            ms = float(np.median(times[label]))
            rows.append(dict(variant=label, log2_words=b, ms=round(ms, 4), mpix_s=round(W * H / 1e6 / (ms / 1e3), 1),
                             vs_hash=round(base / ms, 3), ms_rounds=[round(t, 4) for t in times[label]],
                             radiance_vs_hash=round(energy[label] / energy["hash"], 4)))
            print(f"{name[:28]:28s} {label:22s} {ms:8.3f} ms {rows[-1]['mpix_s']:9.1f} Mpixel/s "
                  f"x{rows[-1]['vs_hash']:.3f} of hash  frame radiance x{rows[-1]['radiance_vs_hash']:.4f}",
                  file=sys.stderr, flush=True)
        result["frames"].append(dict(frame=name, width=W, height=H, rows=rows))
        del dgb, out, ws
    print(json.dumps(result))


if __name__ == "__main__":
    main()
