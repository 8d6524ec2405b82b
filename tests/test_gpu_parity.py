"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Run on an MI355X:  python -u -m pytest tests -m gpu -x -v --timeout 120 --timeout-method thread
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2306_05051_amd import scenes
from parity_util import MARGIN, compare, dbg_to_numpy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hash_vectors.txt")


@pytest.fixture(scope="module")
def glint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_05051_amd import glint as g
    g.lib()
    return g


def _run(glint, gb, mats, lights, **kw):
    print(f"  gpu: {gb['u'].shape} mats={len(mats)} lights={len(lights)} {kw}", flush=True)
    dgb = glint.to_device(gb)
    rgb, dbg = glint.glint_shade(dgb, mats, lights, debug=True, **kw)
    rgb2 = glint.glint_shade(dgb, mats, lights, **kw)
    torch.cuda.synchronize()
    # the production kernel (which skips gates that cannot open and decides
    # small-threshold gates on the hash head) gives the same bits
    assert torch.equal(rgb, rgb2)
    d = dbg_to_numpy(dbg)
    small = d["n_live_small"].astype(np.int64) & 0xFFFFFFFF
    assert np.all(small <= (d["n_live"].astype(np.int64) & 0xFFFFFFFF))
    return rgb.cpu().numpy(), d


def _check(glint, gb, mats, lights, label, min_checked=0.9, **kw):
    grgb, gdbg = _run(glint, gb, mats, lights, **kw)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True, **kw)
    st = compare(grgb, gdbg, rrgb, rdbg, label=label)
    print(f"  {label}: {st}", flush=True)
    # the comparison must not be vacuous: most shaded pixels are compared
    assert st["checked"] > min_checked * st["shaded"]
    return st


def test_hash_vectors_bit_exact(glint):
    steps, texels = [], []
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "step":
            steps.append([int(f[1], 16), int(f[2], 16), int(f[3], 16)])
        else:
            texels.append([int(f[1], 16)] + [int(x) for x in f[2:10]] + [int(f[10], 16)])
    s = np.array(steps, dtype=np.uint64)
    h = torch.from_numpy(s[:, 0].astype(np.uint32).view(np.int32)).cuda()
    w = torch.from_numpy(s[:, 1].astype(np.uint32).view(np.int32)).cuda()
    out = glint.glint_hash_step(h, w).cpu().numpy().view(np.uint32)
    assert np.array_equal(out, s[:, 2].astype(np.uint32))
    t = np.array(texels, dtype=np.int64)
    keys = t[:, :9].copy()
    keys[:, 0] = keys[:, 0].astype(np.uint32).view(np.int32) if False else keys[:, 0]
    k32 = np.empty((len(t), 9), np.int32)
    k32[:, 0] = t[:, 0].astype(np.uint32).view(np.int32)
    k32[:, 1:] = t[:, 1:9].astype(np.int32)
    out = glint.glint_texel_hash(torch.from_numpy(k32).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(out, t[:, 9].astype(np.uint32))


def test_inverse_cdf_accuracy_all_uniforms(glint):
    from scipy.special import ndtri
    k = np.arange(2**23, dtype=np.int64)
    bits = torch.from_numpy(((k << 9) | 0x155).astype(np.uint32).view(np.int32)).cuda()
    z = glint.glint_ndtri(bits).cpu().numpy().astype(np.float64)
    q = (2.0 * k + 1.0) * 2.0**-24
    ref = ndtri(q)
    err = np.abs(z - ref) / np.maximum(np.abs(ref), 1.0)
    print("  max err", err.max(), "at q", q[err.argmax()])
    assert err.max() < 1e-6


@pytest.mark.parametrize("tilt", [0.0, 45.0, 80.0])
def test_plane_256(glint, tilt):
    gb, mats, lights = scenes.plain_forward(256, 256, tilt_deg=tilt, seed=int(tilt))
    _check(glint, gb, mats, lights, f"plane tilt {tilt}")


def test_plane_256_brighter(glint):
    # light placed near the mirror direction so that many gates open
    gb, mats, lights = scenes.plain_forward(256, 256, tilt_deg=30.0, seed=1)
    lights = [dict(dir=(0.0, 0.45, 0.89), radiance=(1.0, 0.8, 0.6))]
    mats = [dict(mats[0], log10_density=7.0)]
    st = _check(glint, gb, mats, lights, "plane bright")
    assert st["nonzero"] > 1000


def test_sphere_scattered_anisotropy(glint):
    gb, mats, lights = scenes.sphere_forward(320, 180, seed=1)
    _check(glint, gb, mats, lights, "sphere 320x180")


def test_sphere_geometric_footprints(glint):
    gb, mats, lights = scenes.sphere_forward(256, 160, seed=2, redraw=False)
    _check(glint, gb, mats, lights, "sphere geometric")


def test_four_k_like_small(glint):
    gb, mats, lights = scenes.four_k(256, 144, seed=3)
    st = _check(glint, gb, mats, lights, "4k-like 256x144")


@pytest.mark.parametrize("view", ["plane90", "plane25", "scattered"])
@pytest.mark.parametrize("k_max,log10_density", [(4, 5.0), (0, 7.0)])
def test_paper_setting_beckmann(glint, view, k_max, log10_density):
    """The paper's performance setting: Beckmann alpha = 1.0 (p clamped to 1
    where R D(h)/D(n) exceeds it), one light, plane views and scattered
    anisotropy; the isotropic family (K = 0) splits every anisotropic
    footprint."""
    gb, mats, lights = scenes.paper_setting(192, 108, view=view, log10_density=log10_density, seed=2)
    # dense, broad-lobed flakes open hundreds of gates per pixel, so more
    # pixels hold a count within 1e-5 of a rounding boundary (excluded, counted)
    _check(glint, gb, mats, lights, f"{view} K={k_max} logN={log10_density}", min_checked=0.75, k_max=k_max)


@pytest.mark.parametrize("view", ["plane90", "plane25"])
def test_p_clamp_flag(glint, view):
    """Eq. 4's p = R D(h)/D(n) exceeds 1 for Beckmann alpha = 1 (up to 1.47 R)
    once R is above 0.68 (reading S15: p clamped to 1, flag bit 2).  With
    R = 0.8 a band of half-vector angles is clamped (13-52% of the pixels in
    these views); the flag, compared wherever no decision sits within the
    margin of its boundary, and the counts (every gate of a clamped light
    opens) follow the oracle on both sides of the band's edges."""
    gb, mats, lights = scenes.paper_setting(192, 108, view=view, log10_density=4.0, seed=3)
    mats = [dict(mats[0], R=0.8)]
    st = _check(glint, gb, mats, lights, f"p clamp {view}", min_checked=0.6)
    assert 0.1 * st["shaded"] < st["p_clamped"] < 0.9 * st["shaded"], st


def test_maximum_materials_and_lights(glint):
    """The largest parameter blocks the ABI takes: 32 materials, 16 lights."""
    gb, mats, lights = scenes.four_k(160, 96, seed=8, n_mat=32, n_light=16)
    assert len(mats) == glint.GLINT_MAX_MATERIALS and len(lights) == glint.GLINT_MAX_LIGHTS
    _check(glint, gb, mats, lights, "32 materials, 16 lights")


@pytest.mark.parametrize("n_light", [2, 3, 4, 5])
def test_two_lanes_per_item_in_short_batches(glint, n_light):
    """A tile's last batch of at most 32 (16) items runs each item on two
    (four, with more than two lights) lanes, lane r taking the lights
    l = r mod 2 (4); the radiance chain keeps light order, so the image
    equals the instrumented kernel's (one lane per item) bit for bit, also
    when the lights do not fill the last group.  The lit masks of
    glint_shade_lit equal the instrumented kernel's per-light counts."""
    gb, mats, lights = scenes.four_k(200, 90, seed=12, n_light=n_light)
    grgb, gdbg = _run(glint, gb, mats, lights)
    H, W = gb["u"].shape
    TW, TH = glint.GLINT_TILE_W, glint.GLINT_TILE_H
    npr = np.zeros(((H + TH - 1) // TH * TH, (W + TW - 1) // TW * TW), np.int64)
    npr[:H, :W] = gdbg["n_probe"]
    S = npr.reshape(npr.shape[0] // TH, TH, npr.shape[1] // TW, TW).sum((1, 3)).ravel()
    last = (S - 1) % 64
    short = int(np.sum((S > 0) & (last < 32)))
    quad = int(np.sum((S > 0) & (last < 16)))
    print(f"  tiles with a last batch of <= 32 (16) items: {short} ({quad}) of {int(np.sum(S > 0))}", flush=True)
    assert short > 20 and quad > 10 and np.sum(S > 64) > 20
    _check(glint, gb, mats, lights, f"short batches, {n_light} lights")
    dgb = glint.to_device(gb)
    rgb_l, lit, probes = glint.glint_shade_lit(dgb, mats, lights, rounding=0)
    torch.cuda.synchronize()
    assert np.array_equal(rgb_l.cpu().numpy(), grgb)
    lit = lit.cpu().numpy().astype(np.int64) & 0xFFFF
    want = sum(((gdbg["b_light"][l] > 0).astype(np.int64) << l) for l in range(n_light))
    assert np.array_equal(lit, want)
    # probe bits only below the pixel's probe count (bit 31: probe 31 or later), set iff a light is lit
    pm = probes.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    npx = gdbg["n_probe"].astype(np.int64)
    assert np.all((pm & ~((1 << np.minimum(npx, 32)) - 1)) == 0)
    assert np.array_equal(pm != 0, lit != 0)


@pytest.mark.parametrize("k_max,n_probe_max", [(0, 21), (1, 21), (2, 8), (4, 1), (3, 64)])
def test_grid_family_variants(glint, k_max, n_probe_max):
    gb, mats, lights = scenes.four_k(96, 80, seed=5, n_light=2)
    _check(glint, gb, mats, lights, f"K={k_max} nmax={n_probe_max}", k_max=k_max, n_probe_max=n_probe_max)


def test_relaxed_counts(glint):
    gb, mats, lights = scenes.four_k(128, 72, seed=6, n_light=3)
    fields = ("n_probe", "level", "cell", "key_sum", "akey_sum", "theta_sum", "n_open", "n_gate")
    grgb, gdbg = _run(glint, gb, mats, lights, rounding=1)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True, rounding=1)
    st = compare(grgb, gdbg, rrgb, rdbg, exact_fields=fields, label="relaxed")
    print(" ", st)


def test_ragged_and_invalid_pixels(glint):
    gb, mats, lights = scenes.ragged_plane(37, 29, seed=1)
    gb = {k: v.copy() for k, v in gb.items()}
    inside = np.argwhere(gb["material_id"] >= 0)
    (a, b, c, d, e) = [tuple(inside[i]) for i in np.linspace(0, len(inside) - 1, 5).astype(int)]
    gb["u"][a] = np.nan                          # non-finite input
    for k in ("dudx", "dudy", "dvdx", "dvdy"):   # det J = 0
        gb[k][b] = 0.0
    gb["wz"][c] = -1.0; gb["wx"][c] = 0.0; gb["wy"][c] = 0.0   # view below surface
    gb["material_id"][d] = 7                     # >= n_mat
    gb["material_id"][e] = -3                    # skipped
    grgb, gdbg = _run(glint, gb, mats, lights)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True)
    compare(grgb, gdbg, rrgb, rdbg, label="ragged")
    for (y, x), bit in ((a, 8), (b, 8), (c, 16), (d, 64), (e, 32)):
        assert gdbg["flags"][y, x] == bit
        assert np.all(grgb[:, y, x] == 0.0)


def test_no_lights_and_empty(glint):
    gb, mats, lights = scenes.ragged_plane(19, 11, seed=2)
    dgb = glint.to_device(gb)
    out = glint.glint_shade(dgb, mats, [])
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    empty = {k: v[:0] for k, v in dgb.items()}
    out = glint.glint_shade(empty, mats, lights)
    assert out.numel() == 0


@pytest.mark.parametrize("case", ["sphere", "four_k", "plane25_sparse", "plane25", "four_k_K0"])
def test_zk_baseline_law(glint, case):
    """The Zirr-Kaplanyan baseline (GLINT_FLAG_ZK_COUNT: Eq. 15 per texel on
    the node's whole cell, node outputs mixed as in Eq. 7) against the
    oracle's count_law=1: flags, keys, per-texel uniforms, Gaussian draws
    (n_open) and every integer count (count_sum) bit-exact, radiance within
    the bar; the production kernel (which skips nodes whose counts are all
    zero) gives the instrumented kernel's bits."""
    kw = {}
    if case == "sphere":
        gb, mats, lights = scenes.sphere_forward(256, 144, seed=4)
    elif case == "four_k":
        gb, mats, lights = scenes.four_k(192, 108, seed=6)
    elif case == "plane25_sparse":
        gb, mats, lights = scenes.paper_setting(192, 108, view="plane25", log10_density=3.0, seed=2)
    elif case == "plane25":
        gb, mats, lights = scenes.paper_setting(192, 108, view="plane25", log10_density=5.0, seed=2)
    else:
        gb, mats, lights = scenes.four_k(128, 96, seed=9, n_light=3)
        kw = dict(k_max=0)
    grgb, gdbg = _run(glint, gb, mats, lights, count_law=glint.LAW_ZK, **kw)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True, count_law=1, **kw)
    st = compare(grgb, gdbg, rrgb, rdbg, label=f"zk {case}")
    shaded = (rdbg["flags"] & 1) > 0
    trials = int(gdbg["n_live"][shaded].astype(np.int64).sum())
    gauss = int(gdbg["n_open"][shaded].astype(np.int64).sum())
    print(f"  zk {case}: {st}; Bernoulli trials {trials}, Gaussian draws {gauss}", flush=True)
    assert st["checked"] > 0.9 * st["shaded"] and st["nonzero"] > 1000
    # both branches of Eq. 15 run (trials are compared through count_sum)
    assert trials > 0 and gauss > 0
    # and so do the trials drawn, on every compared pixel
    m = shaded & (rdbg["margin_pos"] >= MARGIN)
    assert np.array_equal(gdbg["n_live"][m].astype(np.int64) & 0xFFFFFFFF, rdbg["n_live"][m].astype(np.int64))


def test_zk_baseline_differs_from_the_method(glint):
    """Same grids, texels and uniforms, other counting law: the images differ
    while both match their oracle (guards against a flag that is ignored)."""
    gb, mats, lights = scenes.four_k(96, 64, seed=11)
    dgb = glint.to_device(gb)
    a = glint.glint_shade(dgb, mats, lights)
    b = glint.glint_shade(dgb, mats, lights, count_law=glint.LAW_ZK)
    torch.cuda.synchronize()
    assert not torch.equal(a, b)


def test_zk_baseline_rejected_where_unsupported(glint):
    gb, mats, lights = scenes.ragged_plane(8, 8, seed=3)
    dgb = glint.to_device(gb)
    with pytest.raises(glint.GlintError) as e:
        glint.glint_shade(dgb, mats, lights, rounding=1, count_law=glint.LAW_ZK)
    assert e.value.status == glint.GLINT_EINVAL
    table = glint.glint_rng_table_fill(8, 1)
    with pytest.raises(glint.GlintError) as e:
        glint._shade(dgb, mats, lights, 4, 21, 0, None, False, None, None,
                     (table.data_ptr(), 8, glint.RNG_CACHED), glint.LAW_ZK)
    assert e.value.status == glint.GLINT_EINVAL


def test_bad_arguments_rejected(glint):
    gb, mats, lights = scenes.ragged_plane(8, 8, seed=3)
    dgb = glint.to_device(gb)
    with pytest.raises(glint.GlintError) as e:
        glint.glint_shade(dgb, [dict(mats[0], alpha=-1.0)], lights)
    assert e.value.status == glint.GLINT_EINVAL
    with pytest.raises(glint.GlintError) as e:
        glint.glint_shade(dgb, mats, lights, k_max=5)
    assert e.value.status == glint.GLINT_EINVAL
    with pytest.raises(glint.GlintError) as e:
        glint.glint_shade(dgb, mats, lights * 9)
    assert e.value.status == glint.GLINT_EINVAL


def test_deterministic(glint):
    gb, mats, lights = scenes.four_k(128, 128, seed=7)
    dgb = glint.to_device(gb)
    a = glint.glint_shade(dgb, mats, lights)
    b = glint.glint_shade(dgb, mats, lights)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("W,H", [(645, 363), (640, 363)], ids=["odd_columns", "paired"])
def test_tile_order_is_a_heaviest_first_permutation(glint, W, H):
    """The cost-ordered tile schedule: the order is a permutation of the
    tiles, sorted by cost class (heaviest first, ties in row-major order),
    and the image is bit-identical to the row-major schedule.  Ragged size:
    a partial last count block and partial edge tiles.  With an even number
    of tile columns the two tiles of each pair (columns 2m, 2m + 1: the two
    halves of the same 128-byte lines) share the heavier class, are adjacent
    in the sorted order, and run on workgroups b and b + 8 (one XCD)."""
    gb, mats, lights = scenes.four_k(W, H, seed=5)
    dgb = glint.to_device(gb)
    TW, TH = glint.GLINT_TILE_W, glint.GLINT_TILE_H
    tx, ty = (W + TW - 1) // TW, (H + TH - 1) // TH
    n = tx * ty
    paired = tx % 2 == 0
    nb = glint.glint_shade_workspace_bytes(W, H)
    ws = torch.full((nb,), 0xAB, dtype=torch.uint8, device="cuda")
    print(f"  tile order: {W}x{H}, {n} tiles, paired {paired}, workspace {nb} B", flush=True)
    a = glint.glint_shade(dgb, mats, lights, workspace=ws)
    order = ws[:4 * n].view(torch.int32).cpu().numpy().astype(np.int64)
    b = glint.glint_shade(dgb, mats, lights, workspace=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(np.sort(order), np.arange(n))
    # cost classes from the forward's own probe counts (the schedule uses an
    # FP32 estimate of them, so allow a handful of boundary disagreements)
    _, dbg = glint.glint_shade(dgb, mats, lights, debug=True)
    npr = np.zeros((ty * TH, tx * TW), np.int64)
    npr[:H, :W] = dbg["n_probe"].cpu().numpy()
    S = npr.reshape(ty, TH, tx, TW).transpose(0, 2, 1, 3).reshape(n, 64).sum(1)
    bt = (S + 63) // 64
    cls = np.select([bt < 4, bt < 6, bt < 9, bt < 14], [bt, 4, 5, 6], 7)
    seq_order = order
    if paired:
        pair_cls = np.maximum(cls[0::2], cls[1::2])
        cls = np.repeat(pair_cls, 2)
        # undo the slot mapping: workgroup 16q + r holds sorted position
        # 16q + 2r (r < 8) or 16q + 2(r - 8) + 1 (r >= 8); the last partial
        # group of 16 is not mapped
        w = np.arange(n)
        q, r = w // 16, w % 16
        pos = np.where(r < 8, 16 * q + 2 * r, 16 * q + 2 * (r - 8) + 1)
        pos = np.where(w < (n & ~15), pos, w)
        seq_order = np.empty(n, np.int64)
        seq_order[pos] = order
        # line-mates adjacent in the sorted order and on workgroups b, b + 8
        ev, od = seq_order[0::2], seq_order[1::2]
        assert np.all(ev % 2 == 0) and np.all(od == ev + 1)
        full = (n & ~15)
        wg = np.arange(full).reshape(-1, 16)
        assert np.all(order[wg[:, 8:]] == order[wg[:, :8]] + 1)
    seq = cls[seq_order]
    inversions = int(np.sum(seq[1:] > seq[:-1]))
    print(f"  classes {np.bincount(cls, minlength=8).tolist()}, inversions {inversions}", flush=True)
    assert len(np.unique(cls)) >= 3
    assert inversions <= max(2, n // 500)
    # within a class, tiles keep row-major order (stable sort)
    for c in np.unique(seq):
        idx = seq_order[seq == c]
        assert np.mean(np.diff(idx) > 0) > 0.99


@pytest.mark.parametrize("count_law", [0, 1], ids=["method", "zk_baseline"])
def test_full_4k_sampled_rows(glint, count_law):
    """Full-size 3840x2160 frame in the benchmark's launch configuration (and
    the same frame under the Zirr-Kaplanyan baseline); the oracle recomputes
    sampled rows."""
    gb, mats, lights = scenes.four_k(3840, 2160, seed=3)
    dgb = glint.to_device(gb)
    print(f"  full 4K frame, count law {count_law}", flush=True)
    rgb = glint.glint_shade(dgb, mats, lights, count_law=count_law)
    torch.cuda.synchronize()
    rgb = rgb.cpu().numpy()
    rows = [0, 7, 8, 500, 1079, 1080, 1501, 2159]
    for r in rows:
        sub = {k: v[r:r + 1] for k, v in gb.items()}
        rrgb, rdbg = oracle.shade(sub, mats, lights, debug=True, count_law=count_law)
        ok = ((rdbg["flags"] & 1) > 0) & (rdbg["margin_pos"] >= 1e-5)
        g = rgb[:, r:r + 1].astype(np.float64)
        err = np.abs(g - rrgb)[:, ok]
        assert np.all(err <= 1e-4 * np.abs(rrgb[:, ok])), f"row {r}"
        assert np.all(g[:, ~((rdbg["flags"] & 1) > 0)] == 0)


def test_batched_bit_identical_to_per_view(glint):
    views, mats, lights = scenes.batched_views(n_views=9, seed=1, side_min=40, side_max=300)
    dviews = [glint.to_device(v) for v in views]
    ref = [glint.glint_shade(v, mats, lights) for v in dviews]
    outs = [torch.full((3,) + v["u"].shape, -1.0, device="cuda") for v in dviews]
    plan = glint.GlintPlan(dviews, outs, mats, lights)
    for use_graph in (False, True, True):
        for o in outs:
            o.fill_(-1.0)
        plan.run(use_graph=use_graph)
        torch.cuda.synchronize()
        for a, b in zip(ref, outs):
            assert torch.equal(a, b)
    # persistent workgroups, and one workgroup per tile (blocks_per_cu = 0),
    # eager and replayed from a graph
    for tune in ((16, 4, 2), (64, 1, 4), (32, 2, 1), (32, 2, 0), (8, 8, 0)):
        p2 = glint.GlintPlan(dviews, outs, mats, lights, tune=tune)
        for use_graph in (False, True, True):
            for o in outs:
                o.fill_(-1.0)
            p2.run(use_graph=use_graph)
            torch.cuda.synchronize()
            for a, b in zip(ref, outs):
                assert torch.equal(a, b)
        p2.close()
    plan.close()


def test_batched_more_views_than_a_wave(glint):
    """70 small views (more views than lanes in a wave, 16-72 pixels a side):
    the per-tile and the persistent kernel against per-view glint_shade."""
    views, mats, lights = scenes.batched_views(n_views=70, seed=2, side_min=16, side_max=72)
    dviews = [glint.to_device(v) for v in views]
    ref = [glint.glint_shade(v, mats, lights) for v in dviews]
    outs = [torch.full((3,) + v["u"].shape, -1.0, device="cuda") for v in dviews]
    for tune in ((16, 4, 0), (16, 4, 2)):
        plan = glint.GlintPlan(dviews, outs, mats, lights, tune=tune)
        for o in outs:
            o.fill_(-1.0)
        plan.run(use_graph=False)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref, outs)):
            assert torch.equal(a, b), (tune, i)
        plan.close()
