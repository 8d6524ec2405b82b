"""Benchmark: glint-shaded Mpixel/s at 4K on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-backward] [--no-batched] [--no-c5]

Workload (one step = one forward shading of the whole frame, every step of
the method): synthetic 3840x2160 G-buffer of a unit sphere over a ground
plane, 4 directional lights, 8 GGX materials (roughness 0.02-0.6, density
1e3-1e8 flakes per unit UV area, log-uniform) on a seeded Voronoi material
map, footprints of 12 to 252 texels (30% grazing footprints split into 2-21
probes, clustered in the left half, scattered in the right half).  Inputs are
resident in HBM before timing starts.

Prints ONE JSON line on stdout; progress goes to stderr.  The roofline entry
prices the launch's algorithmic VALU work (costmodel.py: slots at the FP32
issue rate, 78.6 T/s) against the time of one glint_shade call (shading
kernel plus its tile-order pre-pass), measured with HIP events on the launch
stream; roofline_bwd does the same for the adjoint call of the 4K
forward+backward step.  Extra keys: the rate over shaded pixels only, the 4K
forward+backward rate, the batched path on 64 views of 128^2..2048^2 against
64 glint_shade calls on the same stream, and the 1024^2 forward+backward
(the adjoint's configuration), and two further fractions of the forward
call: FP32 FLOP/s over the 157.3 TFLOP/s vector peak and VALU instructions
per clock per SIMD over the rate valu_probe measures (both from the
committed counters while the kernel sources match them).  cpu_baseline
times the FP64 oracle on the host cores (model and thread count stated).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "glint_fwd_4k_counters.txt")


def sources_sha256():
    """SHA-256 over the library's kernel sources, C header and build script
    (its compiler flags shape the kernels too)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_05051_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("glint_") and f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "glint.h"), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_2306_05051_amd", "build.py"), "rb").read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per glint_shade call at 4K from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the kernel
    sources have changed since those counters were taken."""
    import re
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return None
    sha = re.search(r"^sources_sha256: ([0-9a-f]{64})$", txt, re.M)
    val = re.search(r"^traffic_bytes_per_call: (\d+)$", txt, re.M)
    if not (sha and val) or sha.group(1) != sources_sha256():
        return None
    return int(val.group(1))


# v_mul_f32 wavefront instructions per clock per SIMD that valu_probe
# sustains with 16 waves per SIMD (profiles/valu_issue_rates.txt)
PROBE_ISSUE_PER_CLK = 0.452


def recorded_instruction_counts():
    """(VALU wavefront instructions, FP32 FLOP instructions) of one 4K
    shading kernel from the committed counter summary (SQ_INSTS_VALU and
    SQ_INSTS_VALU_FLOPS_FP32: an add, multiply or transcendental counts 1, an
    FMA 2), or None when the kernel sources have changed since."""
    import re
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return None
    sha = re.search(r"^sources_sha256: ([0-9a-f]{64})$", txt, re.M)
    valu = re.search(r"^\s+SQ_INSTS_VALU\s+([0-9.e+]+)$", txt, re.M)
    flops = re.search(r"^\s+SQ_INSTS_VALU_FLOPS_FP32\s+([0-9.e+]+)$", txt, re.M)
    if not (sha and valu and flops) or sha.group(1) != sources_sha256():
        return None
    return float(valu.group(1)), float(flops.group(1))


def other_fractions(kernel_ms):
    """The two further fractions of the forward call: (i) FP32 FLOP/s (64
    lanes per counted instruction, an upper bound: idle lanes do no work)
    over the 157.3 TFLOP/s vector peak; (ii) VALU wavefront instructions per
    clock per SIMD over the rate valu_probe sustains for v_mul_f32 (every
    instruction counted once, so half- and quarter-rate ones make this a
    lower bound).  Both from the committed counters and the live call time."""
    from paper_2306_05051_amd import costmodel
    rec = recorded_instruction_counts()
    if rec is None:
        return None
    valu, flop_inst = rec
    t = kernel_ms / 1e3
    flops = 64.0 * flop_inst / t
    per_clk = valu / (costmodel.CU * costmodel.SIMD_PER_CU * costmodel.CLOCK_HZ * t)
    return {"fp32_flop": {"achieved": round(flops / 1e12, 3), "peak": costmodel.FP32_PEAK_FLOPS / 1e12,
                          "unit": "TFLOP/s", "frac": round(flops / costmodel.FP32_PEAK_FLOPS, 4)},
            "valu_issue": {"achieved": round(per_clk, 4), "peak": PROBE_ISSUE_PER_CLK,
                           "unit": "wave-instructions/clock/SIMD", "frac": round(per_clk / PROBE_ISSUE_PER_CLK, 4),
                           "valu_instructions_per_launch": int(valu)}}


def cpu_baseline(gb, mats, lights, target_s=10.0):
    """The FP64 oracle on the same frame, on the host cores: whole frames,
    repeated until about target_s seconds have elapsed (at most 10 times);
    falls back to an evenly spaced row sample when one frame takes longer."""
    import oracle
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    H, W = gb["u"].shape
    rows = np.linspace(0, H - 1, 16).astype(int)
    sub = {k: np.ascontiguousarray(v[rows]) for k, v in gb.items()}
    t0 = time.perf_counter()
    oracle.shade(sub, mats, lights, n_threads=threads)
    est = (time.perf_counter() - t0) * H / 16
    if est <= target_s:
        reps = int(max(1, min(10, target_s // max(est, 1e-3))))
        log(f"cpu baseline: oracle on the full frame x{reps}, {threads} threads")
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.shade(gb, mats, lights, n_threads=threads)
        dt = (time.perf_counter() - t0) / reps
        n_px, what = H * W, f"full {W}x{H} frame, {reps} repetitions, {dt:.2f} s each"
    else:
        n_rows = int(max(16, target_s / est * H))
        rows = np.linspace(0, H - 1, n_rows).astype(int)
        sub = {k: np.ascontiguousarray(v[rows]) for k, v in gb.items()}
        log(f"cpu baseline: oracle on {n_rows} evenly spaced rows, {threads} threads")
        t0 = time.perf_counter()
        oracle.shade(sub, mats, lights, n_threads=threads)
        dt = time.perf_counter() - t0
        n_px, what = n_rows * W, f"{n_rows} of {H} rows (evenly spaced), {dt:.2f} s"
    # one thread, on an evenly spaced row sample of about a fifth of target_s
    n1 = int(max(8, min(H, target_s / 5.0 / max(est * threads, 1e-6) * H)))
    rows1 = np.linspace(0, H - 1, n1).astype(int)
    sub1 = {k: np.ascontiguousarray(v[rows1]) for k, v in gb.items()}
    t0 = time.perf_counter()
    oracle.shade(sub1, mats, lights, n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(n_px / 1e6 / dt, 4), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": what + "; FP64 C oracle (OpenMP over rows), same G-buffer, materials and lights",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "value_1_thread": round(n1 * W / 1e6 / dt1, 4),
            "sample_1_thread": f"{n1} of {H} rows (evenly spaced), {dt1:.2f} s on one thread"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def timed(stream, fn, reps):
    """mean ms of fn() over reps calls, HIP events on `stream` around them"""
    import torch
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(reps):
        fn()
    s1.record(stream)
    torch.cuda.synchronize()
    return s0.elapsed_time(s1) / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-count", action="store_true", help="skip the instrumented unit-count run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-view timing")
    ap.add_argument("--batched-tune", default=None,
                    help="tile_w,tile_h,blocks_per_cu for the batched path instead of autotuning it")
    ap.add_argument("--no-backward", action="store_true", help="skip the forward+backward timings")
    ap.add_argument("--no-c5", action="store_true", help="skip the 1024^2 forward+backward timing")
    ap.add_argument("--scene-cache", default=None, help="npz file to load the 4K scene from / save it to")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy (HBM byte-counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the shading path would shard by pixels or views with no "
              "exchange (the adjoint with one all-reduce of its partial sums), but no multi-GPU run is "
              "provided.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_05051_amd import costmodel, glint, scenes

    W, H = 3840, 2160
    if args.scene_cache and os.path.exists(args.scene_cache):
        z = np.load(args.scene_cache, allow_pickle=False)
        gb = {k: z[k] for k in z.files}
        _, mats, lights = scenes.four_k(16, 16, seed=3)      # same seeded materials and lights
        log("loaded the 4K scene from", args.scene_cache)
    else:
        log("generating the 4K scene ...")
        gb, mats, lights = scenes.four_k(W, H, seed=3)
        if args.scene_cache:
            np.savez(args.scene_cache, **gb)
    if args.copy_calibration:
        import torch as _t
        a = _t.empty(1 << 28, dtype=_t.float32, device="cuda")     # 1 GiB
        b = _t.empty_like(a)
        b.copy_(a)
        _t.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read, 1073741824 bytes written")
        del a, b
    dgb = glint.to_device(gb)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(glint.glint_shade_workspace_bytes(W, H), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        glint.glint_shade(dgb, mats, lights, out=out, workspace=ws)
    torch.cuda.synchronize()

    units = None
    dbg_np = None
    if not args.no_count:
        _, dbg = glint.glint_shade(dgb, mats, lights, debug=True)
        torch.cuda.synchronize()
        dbg_np = {k: v.cpu().numpy() for k, v in dbg.items()}
        units = costmodel.units_from_debug(dbg_np)
        del dbg
        log("units per launch:", units)

    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev_s[i].record(stream)
        glint.glint_shade(dgb, mats, lights, out=out, workspace=ws)
        ev_e[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(ev_s, ev_e)]
    span_ms = ev_s[0].elapsed_time(ev_e[-1])
    ms_per_step = span_ms / args.steps
    kernel_ms = float(np.mean(kern_ms))
    mpx = W * H / 1e6
    value = mpx / (ms_per_step / 1e3)
    log(f"forward 4K: {ms_per_step:.3f} ms/step (kernel {kernel_ms:.3f} ms, wall {wall / args.steps * 1e3:.3f} ms)"
        f" -> {value:.1f} Mpixel/s")

    extra = {}
    n_shaded = int((gb["material_id"] >= 0).sum())
    extra["shaded_pixels"] = n_shaded
    extra["shaded_mpix_s"] = round(n_shaded / 1e6 / (ms_per_step / 1e3), 2)

    roof = None
    if units is not None:
        slots = costmodel.slots(units)
        achieved = slots / (kernel_ms / 1e3)
        roof = {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(costmodel.VALU_PEAK_SLOTS / 1e12, 3), "unit": "Tslot/s",
                "frac": round(achieved / costmodel.VALU_PEAK_SLOTS, 4), "traffic": recorded_traffic(),
                "kernel": "glint_fwd_kernel<false> + tile-order pre-pass", "kernel_ms": round(kernel_ms, 4),
                "slots_per_launch": int(slots), "units_per_launch": units}
    # two further fractions of the forward call (FP32 FLOP/s, VALU issue
    # rate); roofline.frac (algorithmic slots over the issue peak) is the
    # headline one
    fr = other_fractions(kernel_ms)
    if fr is not None:
        extra["fractions"] = fr

    # forward + backward on the same frame (relaxed counts): the forward records
    # which lights and probes opened a gate, the adjoint skips the rest
    roof_bwd = None
    if not args.no_backward:
        go = torch.randn((3, H, W), device="cuda", dtype=torch.float32)
        wsb = torch.empty(max(1, glint.glint_backward_workspace_bytes(W, H, len(mats), len(lights))),
                          dtype=torch.uint8, device="cuda")
        gbn = {k: v for k, v in dgb.items() if k not in ("alpha_px", "log10_density_px")}
        lit = torch.empty((H, W), dtype=torch.int16, device="cuda")
        probes = torch.empty((H, W), dtype=torch.int32, device="cuda")

        def fwd_lit():
            glint.glint_shade_lit(gbn, mats, lights, out=out, lit=lit, probes=probes, rounding=1, workspace=ws)

        def bwd():
            glint.glint_shade_backward(gbn, mats, lights, go, workspace=wsb, lit=lit, probes=probes)

        fwd_lit(); bwd(); torch.cuda.synchronize()
        n_fb = max(3, args.steps // 2)
        fb_ms = timed(stream, lambda: (fwd_lit(), bwd()), n_fb)
        fwd_lit(); torch.cuda.synchronize()
        bwd_ms = timed(stream, bwd, n_fb)
        full_ms = timed(stream, lambda: (glint.glint_shade(gbn, mats, lights, out=out, rounding=1, workspace=ws),
                                         glint.glint_shade_backward(gbn, mats, lights, go, workspace=wsb)), 3)
        extra["fwd_bwd_mpix_s"] = round(mpx / (fb_ms / 1e3), 2)
        extra["fwd_bwd_ms"] = round(fb_ms, 3)
        extra["bwd_ms"] = round(bwd_ms, 3)
        extra["fwd_bwd_all_gates_ms"] = round(full_ms, 3)
        log(f"forward+backward 4K: {fb_ms:.3f} ms -> {extra['fwd_bwd_mpix_s']} Mpixel/s (adjoint call {bwd_ms:.3f} ms; "
            f"re-evaluating every gate: {full_ms:.3f} ms)")
        if dbg_np is not None:
            bu = costmodel.bwd_units(dbg_np, lit.cpu().numpy(), probes.cpu().numpy())
            bslots = costmodel.slots(bu, costmodel.BWD_COST)
            bach = bslots / (bwd_ms / 1e3)
            roof_bwd = {"bound": "alu", "achieved": round(bach / 1e12, 3),
                        "peak": round(costmodel.VALU_PEAK_SLOTS / 1e12, 3), "unit": "Tslot/s",
                        "frac": round(bach / costmodel.VALU_PEAK_SLOTS, 4), "traffic": None,
                        "kernel": "glint_shade_backward with lit masks (lit-pixel list, glint_bwd_unit_kernel, "
                                  "reductions)", "kernel_ms": round(bwd_ms, 4),
                        "slots_per_launch": int(bslots), "units_per_launch": bu}
            log("adjoint units:", bu)
        del go, wsb, lit, probes

    # the adjoint's own configuration: 1024^2, one material, one light
    if not args.no_c5:
        g5, m5, l5, _, _ = scenes.backward_scene(1024, 1024, seed=5)
        d5 = glint.to_device(g5)
        o5 = torch.empty((3, 1024, 1024), device="cuda")
        lit5 = torch.empty((1024, 1024), dtype=torch.int16, device="cuda")
        pr5 = torch.empty((1024, 1024), dtype=torch.int32, device="cuda")
        go5 = torch.randn((3, 1024, 1024), device="cuda")
        ws5 = torch.empty(max(1, glint.glint_backward_workspace_bytes(1024, 1024, 1, 1)), dtype=torch.uint8,
                          device="cuda")

        def fb5():
            glint.glint_shade_lit(d5, m5, l5, out=o5, lit=lit5, probes=pr5, rounding=1)
            glint.glint_shade_backward(d5, m5, l5, go5, workspace=ws5, lit=lit5, probes=pr5)

        fb5(); torch.cuda.synchronize()
        ms5 = timed(stream, fb5, 10)
        extra["c5_fwd_bwd_ms"] = round(ms5, 4)
        extra["c5_fwd_bwd_mpix_s"] = round(1.048576 / (ms5 / 1e3), 2)
        log(f"forward+backward 1024^2: {ms5:.3f} ms -> {extra['c5_fwd_bwd_mpix_s']} Mpixel/s")
        del d5, o5, lit5, pr5, go5, ws5

    # many views of uneven size in one launch against one glint_shade per view
    if not args.no_batched:
        del out, ws
        views, bm, bl = scenes.batched_views(n_views=64, seed=4)
        dviews = [glint.to_device(v) for v in views]
        del views
        outs = [torch.empty((3,) + v["u"].shape, device="cuda") for v in dviews]
        if args.batched_tune:
            best = tuple(int(x) for x in args.batched_tune.split(","))
            log("batched shape (given)", best)
        else:
            from paper_2306_05051_amd.autotune import autotune
            best, tt = autotune(dviews, outs, bm, bl, reps=1)
            log("autotuned batched shape", best, {k: round(v, 3) for k, v in tt.items()})
        plan = glint.GlintPlan(dviews, outs, bm, bl, tune=best)
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        npx = sum(v["u"].numel() for v in dviews)
        bt = timed(stream, lambda: plan.run(use_graph=True), 5)
        wss = [torch.empty(max(1, glint.glint_shade_workspace_bytes(v["u"].shape[1], v["u"].shape[0])),
                           dtype=torch.uint8, device="cuda") for v in dviews]

        def per_view():
            for v, o, w in zip(dviews, outs, wss):
                glint.glint_shade(v, bm, bl, out=o, workspace=w)

        per_view(); torch.cuda.synchronize()
        st = timed(stream, per_view, 5)
        extra["batched_mpix_s"] = round(npx / 1e6 / (bt / 1e3), 2)
        extra["batched_ms"] = round(bt, 4)
        extra["per_view_mpix_s"] = round(npx / 1e6 / (st / 1e3), 2)
        extra["per_view_ms"] = round(st, 4)
        extra["batched_pixels"] = int(npx)
        extra["batched_tune"] = list(best)
        log(f"batched 64 views ({npx} px): {bt:.3f} ms -> {extra['batched_mpix_s']} Mpixel/s; "
            f"64 glint_shade calls {st:.3f} ms -> {extra['per_view_mpix_s']} Mpixel/s")
        plan.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(gb, mats, lights)

    rec = {
        "metric": "glint-shaded Mpixel/s at 4K (fwd, fwd+bwd) + % of FP32 VALU peak",
        "value": round(value, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "forward glint shading, 3840x2160 sphere+ground G-buffer, 4 directional "
                               "lights, 8 GGX materials, footprints 12-252 texels (1-21 probes)",
                   "width": W, "height": H, "lights": len(lights), "materials": len(mats),
                   "k_max": 4, "n_probe_max": 21},
        "roofline": roof,
        "roofline_bwd": roof_bwd,
        "cpu_baseline": cpu,
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
