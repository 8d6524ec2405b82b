"""Pins of the oracle's angular grid (Sec. 5.2, Eq. 14) and of its tangent
frame (CPU only).

Eq. 14 spreads the counts of a half vector over the four angular texels
nearest to its orthographic projection, with bilinear weights.  These tests
hold the oracle to that definition from outside:

* the four weights reconstruct the projected half vector from the texel
  centres (a weight given to the wrong texel moves the reconstruction);
* with the half vector's polar angle fixed (so p, F and G are fixed) the
  distributed count of a pixel is, at every point of the angular plane, the
  textbook bilinear blend of its values at the four surrounding texel
  centres (a permuted weight, a wrong texel offset or a wrong centre fails);
* the relaxed count is continuous when the light moves h across an angular
  cell edge in x and in y, and when the footprint moves across an edge of a
  simplex lattice (Sec. 6.2);
* a supplied tangent (reading: made orthogonal to n, b = n x t) rotates the
  angular plane exactly as rotating the view and the light about n does,
  ignores its component along n and its length, and a tangent parallel to n
  invalidates the pixel.
"""
import math

import numpy as np
import pytest

import oracle

R = 0.034


def _pixel(S=1, uv=(0.37, 0.61), J=((2.0e-3, 0.0), (0.0, 2.0e-3)), n=(0.0, 0.0, 1.0), wi=(0.0, 0.0, 1.0),
           t=None):
    g = {k: np.zeros((1, S), np.float32) for k in oracle.PLANES}
    g["u"][:] = uv[0]; g["v"][:] = uv[1]
    g["dudx"][:] = J[0][0]; g["dudy"][:] = J[0][1]
    g["dvdx"][:] = J[1][0]; g["dvdy"][:] = J[1][1]
    g["nx"][:], g["ny"][:], g["nz"][:] = n
    g["wx"][:], g["wy"][:], g["wz"][:] = wi
    g["material_id"] = np.zeros((1, S), np.int32)
    if t is not None:
        g["tx"], g["ty"], g["tz"] = [np.full((1, S), c, np.float32) for c in t]
    return g


def _mat(micro=0.02, logN=7.0, alpha=0.3, seed=11):
    return dict(ndf=0, alpha=alpha, R=R, log10_density=logN, micro_roughness=micro, F0=1.0, seed=seed)


def _b(g, mats, lights, rounding=1):
    _, d = oracle.shade(g, mats, lights, rounding=rounding, debug=True)
    return d["b_light"][0, 0, 0], d


# ---------------------------------------------------------------------------
# the weights themselves: reconstruction of the projected half vector
# ---------------------------------------------------------------------------
def test_angular_weights_reconstruct_projection():
    rng = np.random.default_rng(21)
    for _ in range(3000):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        h = rng.normal(size=3); h /= np.linalg.norm(h)
        t, b = oracle.tangent_frame(n)
        micro = 10.0 ** rng.uniform(-3, 0)
        ai, aj, v = oracle.angular_texels(h, t, b, micro)
        v = np.array(v)
        assert np.all(v >= 0.0) and v.sum() == pytest.approx(1.0, abs=1e-12)
        # texel a = (ai + (a & 1), aj + (a >> 1)) is centred at ((i + 1/2) micro, (j + 1/2) micro)
        cx = np.array([ai + (a & 1) + 0.5 for a in range(4)]) * micro
        cy = np.array([aj + (a >> 1) + 0.5 for a in range(4)]) * micro
        px, py = float(np.dot(h, t)), float(np.dot(h, b))
        assert float(v @ cx) == pytest.approx(px, abs=1e-12 * max(1.0, abs(px) / micro) * micro + 1e-15)
        assert float(v @ cy) == pytest.approx(py, abs=1e-12 * max(1.0, abs(py) / micro) * micro + 1e-15)
        # the lower-left texel holds the point: its cell coordinates lie in [0, 1)
        fx, fy = px / micro - 0.5 - ai, py / micro - 0.5 - aj
        assert -1e-9 <= fx < 1.0 + 1e-9 and -1e-9 <= fy < 1.0 + 1e-9


# ---------------------------------------------------------------------------
# the distributed count is the bilinear blend of its texel-centre values
# ---------------------------------------------------------------------------
SIN_H = 0.3      # sin of the half vector's polar angle: fixes p, F and G


def _at(x, y, logN=7.0, rounding=1, seed=11):
    """Distributed count with the half vector projecting to (x, y) angular cell
    units (texel (i, j) centred at (i + 1/2, j + 1/2)): the polar angle is fixed,
    the azimuth points at (x, y) and the cell size scales the radius."""
    psi = math.atan2(y, x)
    micro = SIN_H / math.hypot(x, y)
    c = math.sqrt(1.0 - SIN_H * SIN_H)
    h = np.array([SIN_H * math.cos(psi), SIN_H * math.sin(psi), c])
    wo = 2.0 * c * h - np.array([0.0, 0.0, 1.0])         # mirror of the view (0, 0, 1) about h
    g = _pixel()
    b, d = _b(g, [_mat(micro=micro, logN=logN, seed=seed)], [dict(dir=tuple(wo), radiance=(1, 1, 1))],
              rounding)
    return b, d


@pytest.mark.parametrize("rounding", [0, 1])
def test_count_is_bilinear_blend_of_texel_centres(rounding):
    I0, J0 = 3, -2
    V = {}
    for i in range(I0, I0 + 5):
        for j in range(J0, J0 + 5):
            V[i, j], d = _at(i + 0.5, j + 0.5, rounding=rounding)
            assert d["flags"][0, 0] & 1
    vals = np.array(list(V.values()))
    # the texel values differ (independent uniforms per angular texel), so a
    # weight given to the wrong texel changes the blend
    assert len(np.unique(np.round(vals, 9))) > 20 and vals.min() > 0.0
    rng = np.random.default_rng(22)
    pts = [(x, y) for x, y in rng.uniform([I0 + 0.5, J0 + 0.5], [I0 + 4.5, J0 + 4.5], (60, 2))]
    # and points on and next to texel-centre lines and cell edges
    pts += [(I0 + 1.5, J0 + 2.2), (I0 + 2.7, J0 + 3.5), (I0 + 2.0, J0 + 1.1), (I0 + 3.3, J0 + 3.0),
            (I0 + 2.0 + 1e-9, J0 + 3.0 - 1e-9)]
    for x, y in pts:
        b, _ = _at(x, y, rounding=rounding)
        ax, ay = x - 0.5, y - 0.5
        i, j = math.floor(ax), math.floor(ay)
        fx, fy = ax - i, ay - j
        ref = ((1 - fx) * (1 - fy) * V[i, j] + fx * (1 - fy) * V[i + 1, j]
               + (1 - fx) * fy * V[i, j + 1] + fx * fy * V[i + 1, j + 1])
        # the light direction is FP32 (h off by ~1e-7, i.e. ~1e-6 cell units)
        assert b == pytest.approx(ref, rel=2e-5), (x, y, b, ref)


# ---------------------------------------------------------------------------
# continuity across angular cell edges as the light moves
# ---------------------------------------------------------------------------
def _light_for(x, y, micro, wi):
    """A light whose half vector with the view wi projects to (x, y) cell units
    on the basis of n = (0, 0, 1)."""
    px, py = x * micro, y * micro
    h = np.array([px, py, math.sqrt(1.0 - px * px - py * py)])
    wi = np.asarray(wi, np.float64) / np.linalg.norm(wi)
    return 2.0 * np.dot(wi, h) * h - wi


@pytest.mark.parametrize("axis", ["x", "y"])
def test_relaxed_count_continuous_across_angular_edges(axis):
    micro = 0.02
    wi = (0.12, -0.2, 0.97)
    rng = np.random.default_rng(23 if axis == "x" else 24)
    checked = 0
    for trial in range(24):
        edge = float(rng.integers(-6, 6))              # ax = k: the lower-left texel changes
        other = float(rng.uniform(-5.0, 5.0))
        vals = []
        for s in (-1.0, 1.0):
            e = edge + 0.5 + s * 2e-5
            x, y = (e, other) if axis == "x" else (other, e)
            wo = _light_for(x, y, micro, wi)
            b, d = _b(_pixel(wi=wi), [_mat(micro=micro, logN=7.5, seed=trial)],
                      [dict(dir=tuple(wo), radiance=(1, 1, 1))])
            vals.append((b, d))
        (ba, da), (bb, db) = vals
        if min(da["margin"][0, 0], db["margin"][0, 0]) < 1e-4 and da["margin_kind"][0, 0] in (8,):
            continue        # a gate sits on its boundary at one of the two points
        if max(abs(ba), abs(bb)) == 0.0:
            continue
        # a jump would be a whole texel's count; the step moves the weights by ~2e-5
        assert abs(ba - bb) <= 2e-3 * max(abs(ba), abs(bb)), (trial, ba, bb)
        checked += 1
    assert checked >= 12


# ---------------------------------------------------------------------------
# continuity across simplex lattice edges as the footprint moves (Sec. 6.2)
# ---------------------------------------------------------------------------
def _f32_around(x):
    """The FP32 values just below and just above x."""
    f = np.float32(x)
    lo = f if float(f) < x else np.nextafter(f, np.float32(-np.inf))
    hi = np.nextafter(lo, np.float32(np.inf))
    return lo, hi


@pytest.mark.parametrize("edge", ["Lx", "Ly", "diagonal"])
def test_relaxed_count_continuous_across_lattice_edges(edge):
    """An isotropic footprint of area 2^l (1 + ts) has two grids, (l, 0, 0) and
    (l + 1, 0, 0) (Eq. 13, Fig. 4's centre); crossing an edge of the finer
    grid's simplex lattice swaps one vertex whose barycentric weight goes to 0
    there, so the relaxed count changes by ~ the FP32 step of u only."""
    l = -20
    side = math.sqrt(2.0 ** l)                          # cell side of grid (l, 0, 0)
    J = ((math.sqrt(1.37 * 2.0 ** l), 0.0), (0.0, math.sqrt(1.37 * 2.0 ** l)))
    rng = np.random.default_rng({"Lx": 31, "Ly": 32, "diagonal": 33}[edge])
    checked = 0
    wo = (-0.21, 0.12, 0.97)
    for trial in range(30):
        # lattice point (Lx, Ly) on the chosen edge; x' = Lx - Ly/2, y' = Ly; uv = side (x', y')
        Ly = float(rng.integers(40, 400)) + rng.uniform(0.05, 0.95)
        Lx = float(rng.integers(40, 400)) + rng.uniform(0.05, 0.95)
        if edge == "Lx":
            Lx = math.floor(Lx)
        elif edge == "Ly":
            Ly = math.floor(Ly)
        else:
            Lx = math.floor(Lx) + (Ly - math.floor(Ly))   # f = g
        # move along u only: in lattice units u enters x' (and so Lx) alone,
        # which crosses the Lx edge and the diagonal; for Ly move along v
        if edge == "Ly":
            v_edge = Ly * side
            u0 = np.float32((Lx - Ly / 2.0) * side)
            pts = [(u0, vv) for vv in _f32_around(v_edge)]
        else:
            v0 = np.float32(Ly * side)
            Ly = float(v0) / side                          # the lattice row the FP32 v sits on
            if edge == "diagonal":
                Lx = math.floor(Lx) + (Ly - math.floor(Ly))
            u_edge = (Lx - Ly / 2.0) * side
            pts = [(uu, v0) for uu in _f32_around(u_edge)]
        res = []
        for (uu, vv) in pts:
            g = _pixel(uv=(uu, vv), J=J, wi=(0.2, -0.1, 0.97))
            res.append(_b(g, [_mat(logN=8.0, seed=trial)], [dict(dir=wo, radiance=(1, 1, 1))]))
        (ba, da), (bb, db) = res
        assert da["cell"][0, 0] == db["cell"][0, 0] and da["n_probe"][0, 0] == 1
        if da["margin_kind"][0, 0] == 8 and min(da["margin"][0, 0], db["margin"][0, 0]) < 1e-4:
            continue
        if max(abs(ba), abs(bb)) == 0.0:
            continue
        # the two points straddle the edge: some texel key changed
        assert da["key_sum"][0, 0] != db["key_sum"][0, 0]
        # one FP32 step of u is ~6e-8 / 1e-3 ~ 1e-4 lattice units at these coordinates
        assert abs(ba - bb) <= 2e-3 * max(abs(ba), abs(bb)), (trial, ba, bb)
        checked += 1
    assert checked >= 15


# ---------------------------------------------------------------------------
# supplied tangents (reading: orthogonalised against n, b = n x t)
# ---------------------------------------------------------------------------
def _rot_z(v, a):
    c, s = math.cos(a), math.sin(a)
    return (c * v[0] - s * v[1], s * v[0] + c * v[1], v[2])


def test_tangent_frame_of_supplied_tangent():
    rng = np.random.default_rng(41)
    for _ in range(500):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        t0 = rng.normal(size=3)
        res = oracle.frame_of_tangent(n, t0)
        assert res is not None
        t, b = (np.array(x) for x in res)
        tp = t0 - np.dot(t0, n) * n
        assert np.allclose(t, tp / np.linalg.norm(tp), atol=1e-14)
        assert np.allclose(b, np.cross(n, t), atol=1e-14)
        # the component along n and the length do not matter
        res2 = oracle.frame_of_tangent(n, 3.7 * t0 + 0.9 * n)
        assert np.allclose(res2[0], t, atol=1e-13) and np.allclose(res2[1], b, atol=1e-13)
    n = np.array([0.0, 0.6, 0.8])
    assert oracle.frame_of_tangent(n, n) is None
    assert oracle.frame_of_tangent(n, 2.0 * n + np.array([0.0, 8e-4, -6e-4])) is None    # sin ~ 5e-4
    assert oracle.frame_of_tangent(n, n + np.array([0.0, 8e-3, -6e-3])) is not None     # sin ~ 1e-2


def test_supplied_tangent_rotates_the_angular_plane():
    """With n = (0, 0, 1), the tangent (cos g, sin g, 0) projects h on
    (<h, R(g) x>, <h, R(g) y>): the same as rotating the view and the light by
    -g with the basis of n.  Keys, counts and the distributed count agree."""
    rng = np.random.default_rng(42)
    checked = 0
    for trial in range(30):
        g = rng.uniform(0.0, 2.0 * math.pi)
        wi = tuple(rng.normal([0.0, 0.0, 1.0], [0.3, 0.3, 0.0]))
        wo = tuple(rng.normal([0.0, 0.0, 1.0], [0.25, 0.25, 0.0]))
        J = ((3e-3, 1e-3), (-0.5e-3, 2e-3))
        mats = [_mat(logN=6.5, seed=trial)]
        ga = _pixel(J=J, wi=wi, t=(math.cos(g), math.sin(g), 0.0))
        ba, da = _b(ga, mats, [dict(dir=wo, radiance=(1, 1, 1))], rounding=0)
        gb = _pixel(J=J, wi=_rot_z(wi, -g))
        bb, db = _b(gb, mats, [dict(dir=_rot_z(wo, -g), radiance=(1, 1, 1))], rounding=0)
        if min(da["margin_pos"][0, 0], db["margin_pos"][0, 0]) < 1e-4:
            continue
        for k in ("akey_sum", "key_sum", "theta_sum", "count_sum", "n_open"):
            assert da[k][0, 0] == db[k][0, 0], (trial, k)
        assert ba == pytest.approx(bb, rel=1e-5, abs=1e-12)
        checked += 1
    assert checked >= 20
    # a non-unit tangent with a component along n gives the same frame
    ga2 = _pixel(J=J, wi=wi, t=(2.5 * math.cos(g), 2.5 * math.sin(g), 0.8))
    bc, dc = _b(ga2, mats, [dict(dir=wo, radiance=(1, 1, 1))], rounding=0)
    assert dc["akey_sum"][0, 0] == da["akey_sum"][0, 0] and bc == pytest.approx(ba, rel=1e-6, abs=1e-12)


def test_onb_tangent_reproduces_the_default_frame():
    rng = np.random.default_rng(43)
    n = rng.normal(size=3); n /= np.linalg.norm(n)
    n = n if n[2] > 0 else -n
    t, _ = oracle.tangent_frame(n)
    wi = tuple(n + 0.2 * rng.normal(size=3))
    gb_a = _pixel(n=tuple(n), wi=wi)
    gb_b = _pixel(n=tuple(n), wi=wi, t=tuple(t))
    mats, lights = [_mat(logN=7.0)], [dict(dir=tuple(n + 0.3 * rng.normal(size=3)), radiance=(1, 1, 1))]
    _, da = _b(gb_a, mats, lights, rounding=0)
    _, db = _b(gb_b, mats, lights, rounding=0)
    for k in ("flags", "akey_sum", "key_sum", "theta_sum", "count_sum"):
        assert da[k][0, 0] == db[k][0, 0], k


def test_tangent_parallel_to_normal_invalidates_pixel():
    g = _pixel(n=(0.0, 0.6, 0.8), t=(0.0, 0.6, 0.8))
    rgb, d = oracle.shade(g, [_mat()], [dict(dir=(0.1, 0.5, 0.8), radiance=(1, 1, 1))], debug=True)
    assert d["flags"][0, 0] == oracle.FLAG_BAD_INPUT and np.all(rgb == 0.0)
    g = _pixel(t=(np.nan, 1.0, 0.0))
    rgb, d = oracle.shade(g, [_mat()], [dict(dir=(0.1, 0.5, 0.8), radiance=(1, 1, 1))], debug=True)
    assert d["flags"][0, 0] == oracle.FLAG_BAD_INPUT
