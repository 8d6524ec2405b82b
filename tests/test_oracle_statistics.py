"""Statistical pins of the FP64 oracle (CPU only).

* brute force: explicit stratified flakes with one Bernoulli trial each give
  mean N P p and variance N P p (1-p) (whole cells) or between N P p (1-p)
  and N P p (partial cells); the oracle's distributed count at a
  lattice-aligned point has mean sum_g E[gated(n_g, p)] and variance
  sum_g Var[gated(n_g, p)] (closed form), with sum_g n_g = N P exactly.
* convergence of the glint BRDF to the smooth microfacet BRDF as the flake
  density grows (Sec. 3, Eqs. 5-6).
* continuity of the relaxed count across area levels, ratio / orientation
  cells and the orientation wrap, and identical floor counts (coherence,
  Sec. 1); lattice and angular cell edges are crossed in
  test_oracle_angular.py.
* evaluation count: 4 grids x 3 simplex vertices x 4 angular texels = 48
  gated binomials per probe and light (Sec. 6.2).
* gradients: frozen-branch differences equal free differences wherever no
  branch flips.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_2306_05051_amd import scenes

R = 0.034
MICRO = 0.02


def _single_pixel_gbuf(S, uv, J, n=(0.0, 0.0, 1.0), wi=(0.0, 0.0, 1.0)):
    g = {k: np.zeros((1, S), np.float32) for k in oracle.PLANES}
    g["u"][:] = uv[0]; g["v"][:] = uv[1]
    g["dudx"][:] = J[0][0]; g["dudy"][:] = J[0][1]
    g["dvdx"][:] = J[1][0]; g["dvdy"][:] = J[1][1]
    g["nx"][:], g["ny"][:], g["nz"][:] = n
    g["wx"][:], g["wy"][:], g["wz"][:] = wi
    g["material_id"] = np.arange(S, dtype=np.int32).reshape(1, S)
    return g


def _aniso_J(P, r, phi):
    s0, s1 = math.sqrt(P * r), math.sqrt(P / r)
    c, s = math.cos(phi), math.sin(phi)
    return [[c * s0, -s * s1], [s * s0, c * s1]]


def _light_for_h(hz):
    """Light direction making h project onto an angular cell centre for the view
    (0,0,1) and normal (0,0,1): h = normalize(MICRO/2, MICRO/2, hz)."""
    h = np.array([MICRO / 2, MICRO / 2, hz])
    h /= np.linalg.norm(h)
    wo = 2.0 * h[2] * h - np.array([0.0, 0.0, 1.0])
    return wo, h


@pytest.mark.parametrize("rng_table", [None, (16, 0x5EED)], ids=["hash", "table16"])
@pytest.mark.parametrize("P,r,phi,logN,hz", [
    (3.1e-6, 5.3, 0.7, 7.0, 0.999),
    (7.7e-7, 1.0, 0.0, 8.0, 0.995),
    (1.9e-6, 13.0, 2.9, 8.5, 0.999),
])
def test_distributed_count_statistics(P, r, phi, logN, hz, rng_table):
    """Also with the gate uniforms read from a table of 2^16 words (Sec. 6.3's
    precomputed texture): every pixel of the sample indexes the same table, so
    this checks that the table and its keyed index give independent uniforms."""
    S = 6000
    J = _aniso_J(P, r, phi)
    g = _single_pixel_gbuf(S, (0.0, 0.0), J)
    wo, h = _light_for_h(hz)
    alpha = 0.4
    mats = [dict(ndf=0, alpha=alpha, R=R, log10_density=logN, micro_roughness=MICRO, F0=1.0, seed=s)
            for s in range(S)]
    lights = [dict(dir=tuple(wo), radiance=(1, 1, 1))]
    _, dbg = oracle.shade(g, mats, lights, debug=True, rng_table=rng_table)
    b = dbg["b_light"][0, 0]
    assert np.all(dbg["n_probe"] == 1)
    # trials per node and the success probability
    Pf = abs(float(np.float32(J[0][0])) * float(np.float32(J[1][1]))
             - float(np.float32(J[0][1])) * float(np.float32(J[1][0])))
    fp = oracle.footprint(np.float32(J[0][0]), np.float32(J[1][0]), np.float32(J[0][1]), np.float32(J[1][1]))
    nodes, _, _ = oracle.grid_nodes(fp[0], fp[1], fp[2], 4)
    N = 10.0 ** np.float64(np.float32(logN))
    ng = [w * N * 2.0 ** l for (l, k, m, w) in nodes]
    assert sum(ng) == pytest.approx(N * Pf, rel=1e-12)       # distributed trials = N P
    h32 = np.array([0.0, 0.0, 1.0]) + np.array(wo, np.float32).astype(np.float64) / np.linalg.norm(np.array(wo, np.float32).astype(np.float64))
    h32 /= np.linalg.norm(h32)
    p = R * oracle.ndf(0, alpha, h32[2]) / oracle.ndf(0, alpha, 1.0)
    mom = [bf.gated_moments(n, p) for n in ng]
    mean_pred = sum(m for m, _ in mom)
    var_pred = sum(v for _, v in mom)
    se = math.sqrt(var_pred / S)
    assert abs(b.mean() - mean_pred) < 5 * se, (b.mean(), mean_pred, se)
    assert b.var() == pytest.approx(var_pred, rel=8 * math.sqrt(2.0 / S) + 0.02)
    # the flake model the law targets: mean N P p; the residual is the gated
    # approximation's own bias, which the closed form quantifies
    bias = mean_pred - N * Pf * p
    assert abs(b.mean() - N * Pf * p - bias) < 5 * se


def test_bruteforce_flake_model():
    """Stratified flakes with explicit trials: mean N P p for an arbitrary
    partial-cell footprint, variance sum_t f_t p (1 - f_t p) in
    [N P p (1-p), N P p]."""
    rng = np.random.default_rng(11)
    N, p = 400.0, 0.3
    # rotated ellipse with semi-axes a, b, centred off-grid
    a, b, th, cx, cy = 0.31, 0.12, 0.6, 0.013, 0.029
    def inside(x, y):
        dx, dy = x - cx, y - cy
        u = math.cos(th) * dx + math.sin(th) * dy
        v = -math.sin(th) * dx + math.cos(th) * dy
        return (u / a) ** 2 + (v / b) ** 2 <= 1.0
    box = (cx - a, cx + a, cy - a, cy + a)
    P = math.pi * a * b
    counts = bf.stratified_counts(N, inside, p, 4000, rng, box)
    f = bf.coverage_fractions(N, inside, box, sub=48)
    var_exact = float(np.sum(f * p * (1 - f * p)))
    assert f.sum() / N == pytest.approx(P, rel=2e-3)
    se = math.sqrt(var_exact / counts.size)
    assert abs(counts.mean() - N * P * p) < 5 * se + 0.01
    assert N * P * p * (1 - p) * 0.98 <= var_exact <= N * P * p * 1.02
    assert counts.var() == pytest.approx(var_exact, rel=0.1)


def test_convergence_to_smooth_ndf():
    """Sec. 3, Eqs. 5-6: D_P -> D(h) as the flake count grows; the pixel
    average of L / L_smooth tends to 1 and the spread shrinks like 1/sqrt(N)."""
    gb, mats, lights = scenes.plain_forward(48, 48, tilt_deg=35.0, seed=3)
    lights = [dict(dir=(0.3, -0.4, 0.866), radiance=(1.0, 1.0, 1.0))]
    wo = np.array(lights[0]["dir"], np.float32).astype(np.float64); wo /= np.linalg.norm(wo)
    live = gb["material_id"] >= 0
    for kind in (0, 1):
        spreads = []
        for logN in (9.0, 11.0):
            m = [dict(mats[0], ndf=kind, alpha=0.5, log10_density=logN)]
            rgb, dbg = oracle.shade(gb, m, lights, debug=True)
            wi = np.stack([gb["wx"], gb["wy"], gb["wz"]], -1).astype(np.float64)
            wi /= np.linalg.norm(wi, axis=-1, keepdims=True)
            h = wi + wo; h /= np.linalg.norm(h, axis=-1, keepdims=True)
            ci, co, ch = wi[..., 2], wo[2], h[..., 2]
            D = np.vectorize(lambda c: oracle.ndf(kind, 0.5, c))(ch)
            G = 1.0 / (1.0 + np.vectorize(lambda c: oracle.smith_lambda(kind, 0.5, c))(ci)) / \
                (1.0 + oracle.smith_lambda(kind, 0.5, co))
            Ls = D * G / (4.0 * ci)
            ratio = rgb[0][live] / Ls[live]
            assert abs(ratio.mean() - 1.0) < 3e-3, (kind, logN, ratio.mean())
            spreads.append(ratio.std())
        assert spreads[1] < spreads[0] / 5.0


def _one_pixel(J, uv, logN=6.0, rounding=1, seed=7, alpha=0.3):
    g = _single_pixel_gbuf(1, uv, J, wi=(0.2, -0.1, 0.97))
    g["material_id"][:] = 0
    mats = [dict(ndf=0, alpha=alpha, R=R, log10_density=logN, micro_roughness=MICRO, F0=1.0, seed=seed)]
    lights = [dict(dir=(-0.21, 0.12, 0.97), radiance=(1, 1, 1))]
    rgb, dbg = oracle.shade(g, mats, lights, rounding=rounding, debug=True)
    return dbg["b_light"][0, 0, 0], dbg


def test_pixel_continuity_across_boundaries():
    """The relaxed distributed count is continuous across an area level, a
    ratio level, an orientation cell edge and the orientation wrap at pi."""
    eps = 1e-9
    rng = np.random.default_rng(12)
    checked = 0
    for trial in range(40):
        uv = tuple(rng.uniform(0.1, 0.9, 2))
        l = int(rng.integers(-20, -14))
        r = 2.0 ** rng.uniform(0.2, 3.8)
        phi = rng.uniform(0.05, math.pi - 0.05)
        logN = rng.uniform(-l * math.log10(2) + 0.5, -l * math.log10(2) + 2.0)
        cases = [
            (_aniso_J(2.0**l * (1 - eps), r, phi), _aniso_J(2.0**l * (1 + eps), r, phi)),
            (_aniso_J(3.3 * 2.0**l, 4.0 * (1 - eps), phi), _aniso_J(3.3 * 2.0**l, 4.0 * (1 + eps), phi)),
            (_aniso_J(3.3 * 2.0**l, r, math.pi / 4 - eps), _aniso_J(3.3 * 2.0**l, r, math.pi / 4 + eps)),
            (_aniso_J(3.3 * 2.0**l, r, eps), _aniso_J(3.3 * 2.0**l, r, math.pi - eps)),
        ]
        for Ja, Jb in cases:
            ba, da = _one_pixel(Ja, uv, logN)
            bb, db = _one_pixel(Jb, uv, logN)
            if min(da["margin"][0, 0], db["margin"][0, 0]) < 1e-6 and \
                    da["margin_kind"][0, 0] in (8, 9):      # a gate sits on its boundary
                continue
            assert abs(ba - bb) <= 1e-4 * max(1.0, abs(ba)), (trial, ba, bb)
            checked += 1
    assert checked > 100


def test_floor_counts_identical_across_level_boundary():
    rng = np.random.default_rng(13)
    same = 0
    for trial in range(30):
        uv = tuple(rng.uniform(0.1, 0.9, 2))
        l = int(rng.integers(-20, -14))
        phi, r = rng.uniform(0.05, 3.0), 2.0 ** rng.uniform(0.2, 3.8)
        logN = -l * math.log10(2) + 1.5
        ba, da = _one_pixel(_aniso_J(2.0**l * (1 - 1e-12), r, phi), uv, logN, rounding=0)
        bb, db = _one_pixel(_aniso_J(2.0**l * (1 + 1e-12), r, phi), uv, logN, rounding=0)
        assert da["count_sum"][0, 0] == db["count_sum"][0, 0]
        assert ba == pytest.approx(bb, rel=1e-6, abs=1e-9)
        same += 1
    assert same == 30


def test_evaluation_count_48_per_probe_and_light():
    gb, mats, lights = scenes.four_k(96, 64, seed=1, n_light=2)
    _, d = oracle.shade(gb, mats, lights, debug=True)
    sh = (d["flags"] & 1) > 0
    n_nodes = (d["cell"] >> 15) & 7
    lv = d["akey_sum"]  # nonzero whenever at least one light is valid
    # gates per pixel = n_probe * valid_lights * n_nodes * 3 * 4
    per = d["n_gate"][sh] / (d["n_probe"][sh] * n_nodes[sh] * 12)
    assert np.all(np.isin(per, [0, 1, 2]))
    full = sh & (n_nodes == 4)
    assert np.any(full)
    assert np.all(d["n_gate"][full] % 48 == 0)
    assert np.any(d["n_probe"][sh] > 1)


def test_frozen_gradient_equals_free_differences():
    gb, mats, lights, _, _ = scenes.backward_scene(40, 40, seed=2)
    rng = np.random.default_rng(14)
    go = rng.normal(size=(3,) + gb["u"].shape)
    ga, gn, gd, flip_f = oracle.grad(gb, mats, lights, go, step=1e-6, frozen=True)
    ga2, gn2, gd2, flip = oracle.grad(gb, mats, lights, go, step=1e-6, frozen=False)
    # free differences exclude pixels whose branches flip; recompute the frozen
    # gradient on the same pixel set by zeroing their upstream gradient
    go_m = go * (flip == 0)[None]
    ga3, gn3, gd3, _ = oracle.grad(gb, mats, lights, go_m, step=1e-6, frozen=True)
    assert flip.mean() < 0.05
    for a, b in ((ga3, ga2), (gn3, gn2), (gd3, gd2)):
        assert np.allclose(a, b, rtol=1e-5, atol=1e-7 * np.abs(a).max()), (a, b)
    # step refinement: O(h^2) central differences agree across steps
    ga4, gn4, gd4, _ = oracle.grad(gb, mats, lights, go, step=1e-5, frozen=True)
    for a, b in ((ga, ga4), (gn, gn4), (gd, gd4)):
        assert np.allclose(a, b, rtol=1e-6, atol=1e-9 * np.abs(a).max())


def _tangent_planes(gb, seed):
    rng = np.random.default_rng(seed)
    H, W = gb["u"].shape
    t = rng.normal(size=(3, H, W))
    g = dict(gb)
    g["tx"], g["ty"], g["tz"] = [t[i].astype(np.float32) for i in range(3)]
    return g


@pytest.mark.parametrize("case", ["four_k", "per_pixel_alpha_N", "beckmann_clamped", "tangents"])
def test_dual_number_gradient_equals_frozen_differences(case):
    """Two independent routes to the adjoint's gradient: forward-mode
    derivatives (dual numbers through the relaxed forward) and central
    differences with every branch frozen.  They agree to the differences'
    truncation (O(h^2), rtol 1e-5), and the dual route's value part equals
    the relaxed forward's loss.  Cases: 8 GGX materials and 4 lights with
    split footprints; per-pixel roughness and density; Beckmann alpha = 1
    with p clamped at 1 on part of the frame; supplied tangent planes."""
    if case == "four_k":
        gb, mats, lights = scenes.four_k(72, 48, seed=3)
    elif case == "per_pixel_alpha_N":
        gb, mats, lights = scenes.sphere_forward(64, 48, seed=2)
    elif case == "beckmann_clamped":
        gb, mats, lights = scenes.paper_setting(64, 48, view="plane25", seed=1)
        mats = [dict(mats[0], R=0.8)]
    else:
        gb, mats, lights = scenes.four_k(64, 48, seed=6, n_light=2)
        gb = _tangent_planes(gb, 7)
    rng = np.random.default_rng(21)
    go = rng.normal(size=(3,) + gb["u"].shape)
    ga, gn, gd, loss = oracle.grad_dual(gb, mats, lights, go)
    fa, fn, fd, _ = oracle.grad(gb, mats, lights, go, step=1e-6, frozen=True)
    L = oracle.shade(gb, mats, lights, rounding=1)
    assert loss == pytest.approx(float((go * L).sum()), rel=1e-12, abs=1e-12 * np.abs(go * L).sum())
    for a, b, name in ((ga, fa, "alpha"), (gn, fn, "lnN"), (gd, fd, "dir")):
        scale = np.abs(b).max()
        assert scale > 0.0, name
        assert np.allclose(a, b, rtol=1e-5, atol=1e-7 * scale), (name, a, b)


@pytest.mark.parametrize("case", ["four_k", "per_pixel_alpha_N", "beckmann_clamped"])
def test_dual_number_gradient_equals_free_differences_without_flips(case):
    """Free central differences of the relaxed forward (nothing frozen), on
    the pixels none of whose decisions flips within +-h, against the
    dual-number gradient of that masked loss: within 1e-6 relative (step
    1e-6; observed <= 4e-7, on Beckmann's alpha)."""
    if case == "four_k":
        gb, mats, lights = scenes.four_k(72, 48, seed=3)
    elif case == "per_pixel_alpha_N":
        gb, mats, lights = scenes.sphere_forward(64, 48, seed=2)
    else:
        gb, mats, lights = scenes.paper_setting(64, 48, view="plane25", seed=1)
        mats = [dict(mats[0], R=0.8)]
    go = np.random.default_rng(21).normal(size=(3,) + gb["u"].shape)
    _, _, _, flip = oracle.grad(gb, mats, lights, go, step=1e-6, frozen=False)
    assert flip.mean() < 0.01
    gm = go * (flip == 0)
    fa, fn, fd, _ = oracle.grad(gb, mats, lights, gm, step=1e-6, frozen=False)
    ga, gn, gd, _ = oracle.grad_dual(gb, mats, lights, gm)
    for a, b, name in ((fa, ga, "alpha"), (fn, gn, "lnN"), (fd, gd, "dir")):
        scale = np.abs(b).max()
        assert scale > 0.0, name
        assert np.allclose(a, b, rtol=1e-6, atol=1e-8 * scale), (name, a, b)


def test_lit_plane_follows_open_gates():
    """The oracle's per-pixel lit mask (lights with an open gate) agrees with its
    open-gate count and with the distributed counts it produced."""
    gb, mats, lights = scenes.four_k(64, 40, seed=11, n_light=5, n_mat=3)
    _, d = oracle.shade(gb, mats, lights, debug=True)
    lit = d["lit"].astype(np.int64)
    assert np.array_equal(lit != 0, d["n_open"] > 0)
    assert np.all(lit < (1 << len(lights)))
    for l in range(len(lights)):
        has = (lit >> l) & 1
        assert np.all(has[d["b_light"][l] > 0] == 1)
    assert np.count_nonzero(lit) > 50
    gb1, mats1, lights1 = scenes.four_k(48, 24, seed=2, n_light=1, n_mat=2)
    _, d1 = oracle.shade(gb1, mats1, lights1, debug=True)
    assert np.array_equal(d1["lit"], (d1["n_open"] > 0).astype(np.uint32))
