"""The method's counting law against the Zirr-Kaplanyan baseline it replaces.

    python -m paper_2306_05051_amd.law_ablation [--steps 10] [--rounds 2]

glint_shade counts flakes with the distributed gated binomial (Eqs. 10,
16-18); with count_law=LAW_ZK (GLINT_FLAG_ZK_COUNT) the same kernel, on the
same grids, texels and hashed uniforms, counts with the prior art instead:
every grid node counts its whole cell with the classical approximation of
Eq. 15 (a floored Gaussian when n p > 5 or n > 16, else up to 16 Bernoulli
trials) and the node outputs are mixed linearly (Eq. 7).  This times both
laws, alternating them over several rounds (HIP events on the launch stream,
tile-order pass included), on the 4K frame of the benchmark and on the
paper's performance setting (1920x1080, Beckmann alpha = 1.0, one light;
plane views and scattered anisotropy; K in {0, 4}; flake densities 10^3 ...
10^8), and reports per configuration the rate of each law, and for the
baseline its work from one instrumented run: Gaussian draws and Bernoulli
trials per pixel, and the mean over the library's tiles of the tile's largest trial
count (a wave waits for its slowest lane).  Prints one JSON object on stdout
and a table on stderr.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

DENSITIES = (3.0, 4.0, 5.0, 6.0, 7.0, 8.0)
K_LEVELS = (0, 4)


def _tile_max_mean(a, tw=16, th=4):
    H, W = a.shape
    Hp, Wp = (H + th - 1) // th * th, (W + tw - 1) // tw * tw
    b = np.zeros((Hp, Wp), np.float64)
    b[:H, :W] = a
    return float(b.reshape(Hp // th, th, Wp // tw, tw).max(axis=(1, 3)).mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--no-4k", action="store_true")
    ap.add_argument("--only-4k", action="store_true")
    args = ap.parse_args()

    import torch
    from . import glint, scenes

    laws = (("distributed", glint.LAW_DISTRIBUTED), ("zk", glint.LAW_ZK))
    stream = torch.cuda.current_stream()

    def measure(dgb, mats, lights, k, out, ws):
        times = {name: [] for name, _ in laws}
        for _ in range(args.rounds):
            for name, law in laws:
                for _ in range(args.warmup):
                    glint.glint_shade(dgb, mats, lights, k_max=k, out=out, workspace=ws, count_law=law)
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                for _ in range(args.steps):
                    glint.glint_shade(dgb, mats, lights, k_max=k, out=out, workspace=ws, count_law=law)
                s1.record(stream)
                torch.cuda.synchronize()
                times[name].append(s0.elapsed_time(s1) / args.steps)
        res = {}
        for name, law in laws:
            glint.glint_shade(dgb, mats, lights, k_max=k, out=out, workspace=ws, count_law=law)
            res[name + "_energy"] = float(out.double().sum())
            ms = float(np.median(times[name]))
            res[name + "_ms"] = round(ms, 4)
        _, dbg = glint.glint_shade(dgb, mats, lights, k_max=k, debug=True, count_law=glint.LAW_ZK)
        shaded = (dbg["flags"] & 1).bool()
        trials = (dbg["n_live"].double() * shaded).cpu().numpy()
        gauss = (dbg["n_open"].double() * shaded).cpu().numpy()
        ns = max(1, int(shaded.sum()))
        res.update(zk_trials_per_px=round(float(trials.sum()) / ns, 2), zk_trials_max=int(trials.max()),
                   zk_tile_max_trials=round(_tile_max_mean(trials), 2),
                   zk_gauss_per_px=round(float(gauss.sum()) / ns, 2))
        return res

    result = {"rows": []}
    frames = []
    if not args.no_4k:
        gb, mats, lights = scenes.four_k()
        frames.append(("4k", None, None, gb, mats, lights, (4,)))
    W, H = args.width, args.height
    for view in (() if args.only_4k else scenes.PAPER_VIEWS):
        gb, _, lights = scenes.paper_setting(W, H, view=view, log10_density=5.0)
        for d in DENSITIES:
            _, mats, _ = scenes.paper_setting(16, 16, view=view, log10_density=d)
            frames.append((view, d, None, gb, mats, lights, K_LEVELS))
    last_gb, dgb = None, None
    for view, d, _, gb, mats, lights, ks in frames:
        Hf, Wf = gb["u"].shape
        if gb is not last_gb:
            dgb = glint.to_device(gb)
            out = torch.empty((3, Hf, Wf), dtype=torch.float32, device="cuda")
            ws = torch.empty(max(1, glint.glint_shade_workspace_bytes(Wf, Hf)), dtype=torch.uint8, device="cuda")
            last_gb = gb
        for k in ks:
            r = measure(dgb, mats, lights, k, out, ws)
            mp = {n: round(Wf * Hf / 1e6 / (r[n + "_ms"] / 1e3), 1) for n, _ in laws}
            row = dict(view=view, log10_density=d, k_max=k, width=Wf, height=Hf,
                       distributed_mpix_s=mp["distributed"], zk_mpix_s=mp["zk"],
                       zk_vs_distributed=round(mp["zk"] / mp["distributed"], 3),
                       radiance_zk_vs_distributed=round(r["zk_energy"] / r["distributed_energy"], 4),
                       **{k2: v for k2, v in r.items() if k2.startswith("zk_") or k2.endswith("_ms")})
            result["rows"].append(row)
            print(f"{view:9s} logN={d if d is not None else '-':>4} K={k}: distributed {mp['distributed']:9.1f}  "
                  f"zk {mp['zk']:9.1f} Mpixel/s (x{row['zk_vs_distributed']:.3f}); zk per px: "
                  f"{row['zk_gauss_per_px']:.1f} Gaussian, {row['zk_trials_per_px']:.1f} trials "
                  f"(tile max {row['zk_tile_max_trials']:.1f}, max {row['zk_trials_max']}); "
                  f"radiance zk/dist {row['radiance_zk_vs_distributed']:.4f}", file=sys.stderr, flush=True)
    summary = []
    for view in (() if args.only_4k else scenes.PAPER_VIEWS):
        for k in K_LEVELS:
            rs = [x for x in result["rows"] if x["view"] == view and x["k_max"] == k]
            e = {}
            for n in ("distributed", "zk"):
                v = [x[n + "_mpix_s"] for x in rs]
                e[n] = dict(min_mpix_s=min(v), max_mpix_s=max(v), spread=round(max(v) / min(v), 3))
            summary.append(dict(view=view, k_max=k, **e))
    result["summary"] = summary
    print(json.dumps(result))


if __name__ == "__main__":
    main()
