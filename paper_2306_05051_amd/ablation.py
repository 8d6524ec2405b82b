"""Grid-family ablation in the paper's performance setting.

    python -m paper_2306_05051_amd.ablation [--steps 10] [--warmup 2]

For each view of scenes.paper_setting (a plane seen straight down, at 25
degrees, and scattered anisotropy), each largest ratio level K in {0, 1, 2,
4} (K = 0 is the isotropic family: every anisotropic footprint is split into
probes) and each flake density 10^3 ... 10^8 per unit UV area, times
glint_shade on a 1920x1080 frame (Beckmann alpha = 1.0, one light) with HIP
events and reports Mpixel/s.  Per (view, K) the spread of the rate over the
density sweep is the stability figure the paper's Table 1 reports for its
own shader (as min-max frame times).  Prints one JSON object on stdout and a
table on stderr.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

DENSITIES = (3.0, 4.0, 5.0, 6.0, 7.0, 8.0)
K_LEVELS = (0, 1, 2, 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    args = ap.parse_args()

    import torch
    from . import glint, scenes

    W, H = args.width, args.height
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(1, glint.glint_shade_workspace_bytes(W, H)), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for view in scenes.PAPER_VIEWS:
        gb, _, lights = scenes.paper_setting(W, H, view=view, log10_density=5.0)
        dgb = glint.to_device(gb)
        P, r, _ = scenes.footprint_of(gb)
        shaded = gb["material_id"] >= 0
        for k in K_LEVELS:
            for d in DENSITIES:
                _, mats, _ = scenes.paper_setting(16, 16, view=view, log10_density=d)
                for _ in range(args.warmup):
                    glint.glint_shade(dgb, mats, lights, k_max=k, out=out, workspace=ws)
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                for _ in range(args.steps):
                    glint.glint_shade(dgb, mats, lights, k_max=k, out=out, workspace=ws)
                s1.record(stream)
                torch.cuda.synchronize()
                ms = s0.elapsed_time(s1) / args.steps
                npr = np.clip(np.ceil(r[shaded] / float(1 << k)), 1, 21)
                rows.append(dict(view=view, k_max=k, log10_density=d, ms=round(ms, 4),
                                 mpix_s=round(W * H / 1e6 / (ms / 1e3), 1),
                                 mean_probes=round(float(npr.mean()), 3)))
                print(f"{view:9s} K={k} log10 N={d:.0f}: {ms:7.3f} ms  {rows[-1]['mpix_s']:9.1f} Mpixel/s  "
                      f"{rows[-1]['mean_probes']:.2f} probes/px", file=sys.stderr, flush=True)
    summary = []
    for view in scenes.PAPER_VIEWS:
        for k in K_LEVELS:
            v = [x["mpix_s"] for x in rows if x["view"] == view and x["k_max"] == k]
            summary.append(dict(view=view, k_max=k, min_mpix_s=min(v), max_mpix_s=max(v),
                                spread=round(max(v) / min(v), 3)))
    print(json.dumps({"frame": [W, H], "material": "Beckmann alpha=1.0", "lights": 1,
                      "rows": rows, "summary": summary}))


if __name__ == "__main__":
    main()
