"""Comparison of the HIP path with the FP64 oracle (shared by the GPU tests).

Bar (from the method's exactness claims): texel keys, hash outputs and flake
counts bit-exact, radiance within 1e-4 relative, on every pixel none of whose
discrete decisions sits within (0, 1e-5) of its boundary (the oracle's
margins, in each decision's own units); pixels with such a decision are
counted and reported, not compared.  A decision value lying exactly on its
boundary (margin 0: exact arithmetic on both sides, e.g. an axis-aligned
isotropic footprint) is compared like any other, and does not hide another
decision of the same pixel that is near, but not on, its boundary.
"""
import numpy as np

MARGIN = 1e-5
RTOL = 1e-4

EXACT = ("n_probe", "level", "cell", "key_sum", "akey_sum", "theta_sum", "count_sum", "n_open", "n_gate")


def compare(gpu_rgb, gpu_dbg, ref_rgb, ref_dbg, exact_fields=EXACT, rtol=RTOL, label=""):
    """Returns a dict of statistics; raises AssertionError on a parity failure."""
    gflags = gpu_dbg["flags"].astype(np.uint32)
    rflags = ref_dbg["flags"].astype(np.uint32)
    # every flag but the p <= 1 clamp (bit 2) is decided exactly on both sides
    assert np.array_equal(gflags & ~np.uint32(4), rflags & ~np.uint32(4)), \
        f"{label}: flags differ on {np.count_nonzero(gflags != rflags)} pixels"
    shaded = (rflags & 1) > 0
    ok = shaded & (ref_dbg["margin_pos"] >= MARGIN)
    # the clamp (FP32 R D(h)/D(n) > 1 against FP64) wherever no decision, the
    # clamp's included, is within the margin of its boundary
    bad = ok & ((gflags & 4) != (rflags & 4))
    assert not bad.any(), f"{label}: p-clamp flag differs on {bad.sum()} of {ok.sum()} pixels"
    for k in exact_fields:
        a = gpu_dbg[k].astype(np.int64) & 0xFFFFFFFF
        b = ref_dbg[k].astype(np.int64) & 0xFFFFFFFF
        bad = ok & (a != b)
        assert not bad.any(), (f"{label}: {k} differs on {bad.sum()} of {ok.sum()} pixels, "
                               f"first at {np.argwhere(bad)[:3].tolist()}")
    g = gpu_rgb.astype(np.float64)
    err = np.abs(g - ref_rgb)
    lim = rtol * np.abs(ref_rgb)
    bad = (err > lim)[:, ok]
    worst = float(np.max(err[:, ok] / np.maximum(np.abs(ref_rgb[:, ok]), 1e-300))) if ok.any() else 0.0
    assert not bad.any(), f"{label}: radiance off on {bad.sum()} channel-pixels, worst rel {worst:.3e}"
    # pixels that are not shaded are exactly zero on both sides
    assert np.all(g[:, ~shaded] == 0.0)
    stats = dict(shaded=int(shaded.sum()), checked=int(ok.sum()), near_boundary=int((shaded & ~ok).sum()),
                 worst_rel=worst, nonzero=int((ref_rgb[0] > 0).sum()),
                 p_clamped=int(((rflags & 4) > 0).sum()))
    kinds = ref_dbg["margin_pos_kind"][shaded & ~ok]
    stats["near_boundary_kinds"] = {int(k): int(c) for k, c in zip(*np.unique(kinds, return_counts=True))}
    return stats


def dbg_to_numpy(d):
    return {k: dbg_to_numpy(v) if isinstance(v, dict) else v.cpu().numpy() for k, v in d.items()}


def compare_dump(gpu_dump, ref_dump, ref_dbg, yx, relaxed=False, beta_atol=2e-6, count_rtol=RTOL, label=""):
    """Per-texel dump of sampled pixels: texel keys and gate words bit-exact,
    integer counts exact (relaxed counts within count_rtol), barycentric
    weights within beta_atol (FP32 against FP64), on every sampled pixel that
    is not shaded or none of whose decisions is within MARGIN of its
    boundary.  Returns the number of pixels compared."""
    n = 0
    for s, (y, x) in enumerate(yx):
        shaded = (ref_dbg["flags"][y, x] & 1) > 0
        if shaded and not ref_dbg["margin_pos"][y, x] >= MARGIN:
            continue
        for k in ("key", "theta"):
            a = gpu_dump[k][s].astype(np.int64) & 0xFFFFFFFF
            b = ref_dump[k][s].astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(a, b), f"{label}: dump {k} differs at pixel {(y, x)} ({np.sum(a != b)} entries)"
        gb, rb = gpu_dump["beta"][s].astype(np.float64), ref_dump["beta"][s]
        assert np.all(np.abs(gb - rb) <= beta_atol), f"{label}: beta off at {(y, x)}"
        assert np.array_equal(gb == 0, rb == 0), f"{label}: beta support differs at {(y, x)}"
        gc, rc = gpu_dump["count"][s].astype(np.float64), ref_dump["count"][s]
        assert np.array_equal(gc != 0, rc != 0), f"{label}: open gates differ at {(y, x)}"
        if relaxed:
            assert np.all(np.abs(gc - rc) <= count_rtol * np.abs(rc)), f"{label}: relaxed count off at {(y, x)}"
        else:
            assert np.array_equal(gc, rc), f"{label}: count differs at {(y, x)}"
        n += 1
    return n
