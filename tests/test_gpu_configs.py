"""GPU parity at the benchmark configurations' full sizes and at the ABI's
layout options, through the C ABI:

  * batched: 64 views of 128^2..2048^2 (51.8 Mpx) in one plan with the
    autotuned launch shape, each view bit-identical to glint_shade on it, and
    sampled rows of the smallest, largest and two more views against the
    oracle;
  * forward 1920x1080 with per-pixel roughness and density: every discrete
    decision's fingerprint on sampled rows bit-exact against the oracle;
  * backward 1024x1024: the autograd Function's adjoint against the oracle's
    FP64 frozen-branch gradient (1e-3) and against central differences of the
    GPU's relaxed forward restricted to pixels none of whose decisions flips
    within the step, for roughness, density and the light direction;
  * padded rows (stride > width) through glint_shade, glint_shade_lit and the
    masked adjoint: the same image, masks and gradients as unpadded planes;
  * supplied tangent planes (Sec. 5.2, Eq. 14): parity with the oracle, and
    degenerate tangents flagged invalid on both sides.

Run on an MI355X:  python -u -m pytest tests/test_gpu_configs.py -x -v --timeout 300 --timeout-method thread
"""
import math

import numpy as np
import pytest

import oracle
from paper_2306_05051_amd import scenes
from parity_util import MARGIN, compare, dbg_to_numpy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def glint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_05051_amd import glint as g
    g.lib()
    return g


def _rows_against_oracle(rgb, gb, mats, lights, rows, label, **kw):
    """radiance of the given rows of a GPU image against the oracle (1e-4
    relative on every pixel none of whose decisions sits within the margin of
    its boundary; unshaded pixels exactly 0); returns (checked, shaded)."""
    checked = shaded_n = 0
    for r in rows:
        sub = {k: np.ascontiguousarray(v[r:r + 1]) for k, v in gb.items()}
        rrgb, rdbg = oracle.shade(sub, mats, lights, debug=True, **kw)
        shaded = (rdbg["flags"] & 1) > 0
        ok = shaded & (rdbg["margin_pos"] >= MARGIN)
        g = rgb[:, r:r + 1].astype(np.float64)
        err = np.abs(g - rrgb)[:, ok]
        assert np.all(err <= 1e-4 * np.abs(rrgb[:, ok])), f"{label} row {r}: worst {err.max()}"
        assert np.all(g[:, ~shaded] == 0.0), f"{label} row {r}"
        checked += int(ok.sum())
        shaded_n += int(shaded.sum())
    return checked, shaded_n


def test_batched_64_views_autotuned(glint):
    from paper_2306_05051_amd.autotune import autotune
    views, mats, lights = scenes.batched_views(n_views=64, seed=4)
    npx = sum(v["u"].size for v in views)
    sides = [v["u"].shape[0] for v in views]
    print(f"  64 views, sides {min(sides)}..{max(sides)}, {npx} pixels", flush=True)
    assert len(views) == 64 and min(sides) >= 128 and max(sides) <= 2048 and npx > 40_000_000
    dviews = [glint.to_device(v) for v in views]
    ref = [glint.glint_shade(v, mats, lights) for v in dviews]
    outs = [torch.full((3,) + v["u"].shape, -1.0, device="cuda") for v in dviews]
    best, timings = autotune(dviews, outs, mats, lights, reps=1)
    print(f"  autotuned shape {best}: {timings[best]:.3f} ms per launch", flush=True)
    # the autotuned plan and the persistent kernel, eager and replayed from a graph
    for tune in (best, (32, 2, 8)):
        plan = glint.GlintPlan(dviews, outs, mats, lights, tune=tune)
        for use_graph in (False, True, True):
            for o in outs:
                o.fill_(-1.0)
            plan.run(use_graph=use_graph)
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(ref, outs)):
                assert torch.equal(a, b), f"view {i} ({sides[i]}^2), tune {tune}, graph {use_graph}"
        plan.close()
    # oracle rows on the smallest, the largest and two other views
    order = np.argsort(sides)
    for i in (int(order[0]), int(order[-1]), int(order[20]), int(order[45])):
        s = sides[i]
        rows = sorted({0, s // 3, s // 2 + 1, s - 1})
        rgb = outs[i].cpu().numpy()
        checked, shaded = _rows_against_oracle(rgb, views[i], mats, lights, rows, f"view {i}")
        print(f"  view {i} ({s}^2): {checked} of {shaded} shaded pixels of rows {rows} checked", flush=True)
        assert checked > 0.95 * shaded and shaded > 0


def test_forward_1080p_per_pixel_material_rows(glint):
    gb, mats, lights = scenes.sphere_forward(1920, 1080, seed=1)
    assert "alpha_px" in gb and "log10_density_px" in gb
    dgb = glint.to_device(gb)
    rgb, dbg = glint.glint_shade(dgb, mats, lights, debug=True)
    prod = glint.glint_shade(dgb, mats, lights)
    torch.cuda.synchronize()
    assert torch.equal(rgb, prod)
    rgb = rgb.cpu().numpy()
    d = dbg_to_numpy(dbg)
    rows = [0, 1, 2, 3, 137, 540, 541, 777, 1000, 1078, 1079]
    sub = {k: np.ascontiguousarray(v[rows]) for k, v in gb.items()}
    rrgb, rdbg = oracle.shade(sub, mats, lights, debug=True)
    gsub = {k: np.ascontiguousarray(v[..., rows, :]) for k, v in d.items()}
    st = compare(np.ascontiguousarray(rgb[:, rows]), gsub, rrgb, rdbg, label="1080p rows")
    print(f"  1080p rows: {st}", flush=True)
    assert st["checked"] > 0.95 * st["shaded"] and st["shaded"] > 5000


def _decisions(glint, dgb, mats, lights):
    _, dbg = glint.glint_shade(dgb, mats, lights, rounding=1, debug=True)
    keys = ("flags", "n_probe", "level", "cell", "key_sum", "akey_sum", "theta_sum", "n_open", "n_live")
    return torch.stack([dbg[k].to(torch.int64) for k in keys])


def test_backward_1024(glint):
    from paper_2306_05051_amd.autograd import GlintShade
    gb, mats, lights, tmats, tlights = scenes.backward_scene(1024, 1024, seed=5)
    dgb = glint.to_device(gb)
    Lt = glint.glint_shade(dgb, tmats, tlights, rounding=1)
    a = torch.tensor([mats[0]["alpha"]], dtype=torch.float64, requires_grad=True)
    n = torch.tensor([mats[0]["log10_density"] * math.log(10.0)], dtype=torch.float64, requires_grad=True)
    d = torch.tensor([lights[0]["dir"]], dtype=torch.float64, requires_grad=True)
    L = GlintShade.apply(a, n, d, dgb, mats, lights)
    loss = 0.5 * ((L - Lt).double() ** 2).sum()
    loss.backward()
    g_ad = np.concatenate([a.grad.numpy(), n.grad.numpy(), d.grad.numpy().ravel()])
    print(f"  adjoint {g_ad}", flush=True)
    # the oracle's FP64 gradient of the same loss, branches frozen
    go = (L - Lt).detach().cpu().numpy().astype(np.float64)
    ra, rn, rd, _ = oracle.grad(gb, mats, lights, go, step=1e-6, frozen=True)
    g_or = np.concatenate([ra, rn, rd.ravel()])
    print(f"  oracle  {g_or}", flush=True)
    scale = np.abs(g_or).max()
    assert np.all(np.abs(g_ad - g_or) <= 1e-3 * np.abs(g_or) + 2e-5 * scale), (g_ad, g_or)
    # and its forward-mode dual-number gradient
    ja, jn, jd, _ = oracle.grad_dual(gb, mats, lights, go)
    g_du = np.concatenate([ja, jn, jd.ravel()])
    print(f"  dual    {g_du}", flush=True)
    assert np.all(np.abs(g_ad - g_du) <= 1e-3 * np.abs(g_du) + 2e-5 * scale), (g_ad, g_du)
    # central differences of the GPU's relaxed forward on the pixels none of
    # whose decisions flips within +-h, against the adjoint of that masked loss
    a0, n0 = float(a), float(n)
    d0 = [float(x) for x in d.detach().numpy()[0]]
    base = _decisions(glint, dgb, mats, lights)

    def params(da=0.0, dn=0.0, dd=(0.0, 0.0, 0.0)):
        m = [dict(mats[0], alpha=a0 + da, log10_density=(n0 + dn) / math.log(10.0))]
        lt = [dict(lights[0], dir=tuple(x + y for x, y in zip(d0, dd)))]
        return m, lt

    h = 2e-4
    steps = [dict(da=h), dict(dn=h)] + [dict(dd=tuple(h if c == k else 0.0 for c in range(3))) for k in range(3)]
    keep = torch.ones_like(base[0], dtype=torch.bool)
    for st in steps:
        for sgn in (1.0, -1.0):
            kw = {k: (sgn * v if not isinstance(v, tuple) else tuple(sgn * x for x in v)) for k, v in st.items()}
            m, lt = params(**kw)
            keep &= (_decisions(glint, dgb, m, lt) == base).all(0)
    frac = float(keep.float().mean())
    print(f"  pixels without a decision flip over all steps: {frac:.4f}", flush=True)
    assert frac > 0.9
    mask = keep.float()[None]
    gm = ((L - Lt).detach() * mask).float().contiguous()
    ga, gn, gd = glint.glint_shade_backward(dgb, mats, lights, gm)

    def f(**kw):
        m, lt = params(**kw)
        Lx = glint.glint_shade(dgb, m, lt, rounding=1)
        return 0.5 * float((((Lx - Lt) * mask).double() ** 2).sum())

    fd = []
    for st in steps:
        plus = f(**st)
        minus = f(**{k: (-v if not isinstance(v, tuple) else tuple(-x for x in v)) for k, v in st.items()})
        fd.append((plus - minus) / (2 * h))
    torch.cuda.synchronize()
    g_m = np.concatenate([ga.cpu().numpy(), gn.cpu().numpy(), gd.cpu().numpy().ravel()]).astype(np.float64)
    fd = np.array(fd)
    print(f"  masked adjoint {g_m}\n  central diff.  {fd}", flush=True)
    sc = np.abs(fd).max()
    assert np.all(np.abs(g_m - fd) <= 1e-2 * np.abs(fd) + 1e-3 * sc), (g_m, fd)


def test_padded_stride(glint):
    gb, mats, lights = scenes.four_k(300, 170, seed=17, n_light=3, n_mat=4)
    W = gb["u"].shape[1]
    dense = glint.to_device(gb)
    padded = glint.to_device(gb, stride=W + 37)
    assert padded["u"].stride(0) == W + 37
    a = glint.glint_shade(dense, mats, lights)
    b = glint.glint_shade(padded, mats, lights)
    a_d, da = glint.glint_shade(dense, mats, lights, debug=True)
    b_d, db = glint.glint_shade(padded, mats, lights, debug=True)
    la = glint.glint_shade_lit(dense, mats, lights, rounding=1)
    lb = glint.glint_shade_lit(padded, mats, lights, rounding=1)
    nb = glint.glint_shade_noalloc(padded, mats, lights)
    torch.cuda.synchronize()
    assert b.stride(1) == W + 37
    assert torch.equal(a, b) and torch.equal(a_d, b_d) and torch.equal(a, nb)
    for k in da:
        assert torch.equal(da[k], db[k]), k
    for x, y in zip(la, lb):
        assert torch.equal(x, y)
    assert float(a.abs().sum()) > 0
    go = torch.randn((3,) + gb["u"].shape, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    ga = glint.glint_shade_backward(dense, mats, lights, go, lit=la[1], probes=la[2])
    gb_ = glint.glint_shade_backward(padded, mats, lights, go, lit=lb[1], probes=lb[2])
    gf = glint.glint_shade_backward(padded, mats, lights, go)
    torch.cuda.synchronize()
    for x, y, z in zip(ga, gb_, gf):
        x, y, z = x.double(), y.double(), z.double()
        tol = 1e-5 * float(x.abs().max()) + 1e-30
        assert float((x - y).abs().max()) <= tol and float((x - z).abs().max()) <= tol
    # and against the oracle (which reads the unpadded planes)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True)
    st = compare(b_d.cpu().numpy(), dbg_to_numpy(db), rrgb, rdbg, label="padded")
    print(f"  padded stride: {st}", flush=True)


def _with_tangents(gb, seed, degenerate=True):
    """random tangent planes (not unit length), a few of them degenerate"""
    rng = np.random.default_rng(seed)
    H, W = gb["u"].shape
    t = rng.normal(size=(3, H, W)) * rng.uniform(0.2, 5.0, size=(1, H, W))
    g = dict(gb)
    n = np.stack([gb["nx"], gb["ny"], gb["nz"]]).astype(np.float64)
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    if degenerate:
        live = np.argwhere(gb["material_id"] >= 0)
        pick = live[rng.choice(len(live), 8, replace=False)]
        for q, (y, x) in enumerate(pick):
            if q < 3:      # parallel to n (up to FP32 rounding): no frame
                t[:, y, x] = 2.0 * n[:, y, x]
            elif q < 5:    # zero length
                t[:, y, x] = 0.0
            elif q < 7:    # 1e-4 rad off n: sin^2 = 1e-8 < 1e-6, no frame
                perp = np.cross(n[:, y, x], [0.3, 0.5, 0.8])
                perp /= np.linalg.norm(perp)
                t[:, y, x] = n[:, y, x] + 1e-4 * perp
            else:          # 0.1 rad off n: a valid frame
                perp = np.cross(n[:, y, x], [0.3, 0.5, 0.8])
                perp /= np.linalg.norm(perp)
                t[:, y, x] = n[:, y, x] + 0.1 * perp
    for i, k in enumerate(("tx", "ty", "tz")):
        g[k] = t[i].astype(np.float32)
    return g


def test_tangent_planes_parity(glint):
    gb, mats, lights = scenes.four_k(256, 144, seed=19, n_light=3)
    g = _with_tangents(gb, 1)
    grgb, gdbg = glint.glint_shade(glint.to_device(g), mats, lights, debug=True)
    prod = glint.glint_shade(glint.to_device(g), mats, lights)
    plain = glint.glint_shade(glint.to_device(gb), mats, lights)
    torch.cuda.synchronize()
    assert torch.equal(grgb, prod)
    rrgb, rdbg = oracle.shade(g, mats, lights, debug=True)
    st = compare(grgb.cpu().numpy(), dbg_to_numpy(gdbg), rrgb, rdbg, label="tangents")
    print(f"  tangent planes: {st}", flush=True)
    assert st["checked"] > 0.9 * st["shaded"]
    # the seven degenerate tangents are invalid input on both sides (flags compared above)
    assert int(((gdbg["flags"].cpu().numpy() & 8) > 0).sum()) >= 7
    # the tangent turns the angular grid: a different image from the basis of n
    assert not torch.equal(prod, plain)
    # the adjoint with tangents against the oracle's gradient
    gs, ms, ls, _, _ = scenes.backward_scene(128, 96, seed=8)
    gs = _with_tangents(gs, 2, degenerate=False)
    dgs = glint.to_device(gs)
    go = torch.randn((3,) + gs["u"].shape, device="cuda", generator=torch.Generator("cuda").manual_seed(8))
    _, lit, probes = glint.glint_shade_lit(dgs, ms, ls, rounding=1)
    ga, gn, gd = glint.glint_shade_backward(dgs, ms, ls, go, lit=lit, probes=probes)
    torch.cuda.synchronize()
    ra, rn, rd, _ = oracle.grad(gs, ms, ls, go.cpu().numpy().astype(np.float64), step=1e-6, frozen=True)
    g_ad = np.concatenate([ga.cpu().numpy(), gn.cpu().numpy(), gd.cpu().numpy().ravel()])
    g_or = np.concatenate([ra, rn, rd.ravel()])
    print(f"  adjoint {g_ad}\n  oracle  {g_or}", flush=True)
    assert np.all(np.abs(g_ad - g_or) <= 1e-3 * np.abs(g_or) + 2e-5 * np.abs(g_or).max())
    ja, jn, jd, _ = oracle.grad_dual(gs, ms, ls, go.cpu().numpy().astype(np.float64))
    g_du = np.concatenate([ja, jn, jd.ravel()])
    assert np.all(np.abs(g_ad - g_du) <= 1e-3 * np.abs(g_du) + 2e-5 * np.abs(g_du).max()), (g_ad, g_du)
