"""Seeded synthetic G-buffers shaped like the paper's benchmark scenes.

This module holds only scene geometry (cameras, ray differentials, uv
maps, material maps, lights).  It contains none of the glint method's
arithmetic and is the one input source shared by the HIP path and the
oracle.  All geometry is computed in FP64 with numpy ``PCG64`` generators
and cast to FP32 planes at the end.

Screen-space uv derivatives come from ray differentials (Igehy 1999): for a
hit point X = E + t D on a surface with normal n,
    dX/dx = t (I - D n^T / <D, n>) dD/dx,
and duv/dx = (d uv / dX) dX/dx -- the quantity a rasteriser's ddx/ddy
approximates (the paper reads its footprints from screen-space derivatives,
Sec. 5.1).

Scenes (the paper's Unity scenes and assets are not available; these stand
in for them):
  plane     textured plane z=0 over [-1/2,1/2]^2, uv = (x+1/2, y+1/2), pinhole
            camera at distance 1.5, FOV 40 deg, tilted about x ("Plane 90/25").
  sphere    unit sphere + ground plane y=-1 (uv = (x,z)/4), random camera,
            FOV 60 deg, with grazing ground pixels ("Sphere", "Heightmap"-like).
Footprint redraws keep each pixel's geometric area P and orientation phi and
replace the anisotropy ratio r:  J' = R(phi) diag(sqrt(P r), sqrt(P/r)).
"""
from __future__ import annotations

import math

import numpy as np

PLANES = ("u", "v", "dudx", "dvdx", "dudy", "dvdy", "nx", "ny", "nz", "wx", "wy", "wz")

DEFAULT_R = 0.034          # ratio R printed for matching Chermain et al. (Sec. 7.2)
DEFAULT_MICRO = 0.02       # angular cell size in projected-h units
DEFAULT_F0 = 1.0


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _camera(eye, target, up, fov_deg, W, H):
    """Per-pixel unnormalised ray directions D and their screen derivatives."""
    eye = np.asarray(eye, np.float64)
    f = _normalize(np.asarray(target, np.float64) - eye)
    rt = _normalize(np.cross(f, np.asarray(up, np.float64)))
    upv = np.cross(rt, f)
    th = math.tan(math.radians(fov_deg) / 2.0)
    asp = W / H
    xs = (2.0 * (np.arange(W) + 0.5) / W - 1.0) * th * asp
    ys = (1.0 - 2.0 * (np.arange(H) + 0.5) / H) * th
    D = f[None, None, :] + xs[None, :, None] * rt[None, None, :] + ys[:, None, None] * upv[None, None, :]
    dDdx = (2.0 / W) * th * asp * rt
    dDdy = -(2.0 / H) * th * upv
    return eye, D, dDdx, dDdy


def _differentials(t, D, n, dDdx, dDdy):
    """Ray-differential transfer of dD/dx, dD/dy to the surface (Igehy 1999)."""
    Dn = np.sum(D * n, axis=-1, keepdims=True)
    def transfer(dD):
        dD = np.broadcast_to(dD, D.shape)
        return t[..., None] * (dD - D * np.sum(dD * n, axis=-1, keepdims=True) / Dn)
    return transfer(dDdx), transfer(dDdy)


def _empty(H, W):
    g = {k: np.zeros((H, W), np.float64) for k in PLANES}
    g["nz"][:] = 1.0
    g["wz"][:] = 1.0
    g["dudx"][:] = 1.0
    g["dvdy"][:] = 1.0
    g["material_id"] = np.full((H, W), -1, np.int32)
    return g


def _finish(g):
    out = {k: np.ascontiguousarray(g[k], dtype=np.float32) for k in PLANES}
    out["material_id"] = np.ascontiguousarray(g["material_id"], dtype=np.int32)
    for k in ("alpha_px", "log10_density_px"):
        if g.get(k) is not None:
            out[k] = np.ascontiguousarray(g[k], dtype=np.float32)
    return out


def plane_gbuffer(W, H, tilt_deg, fov_deg=40.0, dist=1.5):
    """Plane z=0, [-1/2,1/2]^2, uv=(x+1/2, y+1/2), camera tilted about x."""
    th = math.radians(tilt_deg)
    eye = (0.0, -dist * math.sin(th), dist * math.cos(th))
    up = (0.0, math.cos(th), math.sin(th))
    E, D, dDdx, dDdy = _camera(eye, (0, 0, 0), up, fov_deg, W, H)
    n = np.array([0.0, 0.0, 1.0])
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -E[2] / D[..., 2]
    X = E + t[..., None] * D
    hit = (t > 0) & (np.abs(X[..., 0]) <= 0.5) & (np.abs(X[..., 1]) <= 0.5)
    g = _empty(H, W)
    nn = np.broadcast_to(n, D.shape)
    dXdx, dXdy = _differentials(t, D, nn, dDdx, dDdy)
    wi = -_normalize(D)
    g["u"] = np.where(hit, X[..., 0] + 0.5, 0.0)
    g["v"] = np.where(hit, X[..., 1] + 0.5, 0.0)
    g["dudx"] = np.where(hit, dXdx[..., 0], 1.0)
    g["dvdx"] = np.where(hit, dXdx[..., 1], 0.0)
    g["dudy"] = np.where(hit, dXdy[..., 0], 0.0)
    g["dvdy"] = np.where(hit, dXdy[..., 1], 1.0)
    g["nx"][:] = 0.0; g["ny"][:] = 0.0; g["nz"][:] = 1.0
    g["wx"], g["wy"], g["wz"] = wi[..., 0], wi[..., 1], wi[..., 2]
    g["material_id"] = np.where(hit, 0, -1).astype(np.int32)
    return g


def sphere_gbuffer(W, H, rng, fov_deg=60.0, ground_extent=40.0):
    """Unit sphere at the origin + ground plane y=-1 from a random camera."""
    h = rng.uniform(0.2, 2.0)
    d = rng.uniform(2.5, 4.0)
    az = rng.uniform(0.0, 2.0 * math.pi)
    eye = (d * math.cos(az), h, d * math.sin(az))
    target = rng.normal(0.0, 0.15, 3) + np.array([0.0, -0.3, 0.0])
    E, D, dDdx, dDdy = _camera(eye, target, (0, 1, 0), fov_deg, W, H)
    g = _empty(H, W)
    # sphere hit
    b = np.sum(D * E, axis=-1)
    a = np.sum(D * D, axis=-1)
    c = np.dot(E, E) - 1.0
    disc = b * b - a * c
    with np.errstate(invalid="ignore", divide="ignore"):
        ts = (-b - np.sqrt(np.maximum(disc, 0.0))) / a
        tp = (-1.0 - E[1]) / D[..., 1]
    hs = (disc > 0) & (ts > 0)
    Xp = E + tp[..., None] * D
    hp = (tp > 0) & (np.abs(Xp[..., 0]) < ground_extent) & (np.abs(Xp[..., 2]) < ground_extent)
    use_s = hs & (~hp | (ts < tp))
    use_p = hp & ~use_s
    wi = -_normalize(D)
    # sphere
    Xs = E + ts[..., None] * D
    ns = _normalize(np.where(use_s[..., None], Xs, np.array([0.0, 1.0, 0.0])))
    dXdx, dXdy = _differentials(np.where(use_s, ts, 1.0), D, ns, dDdx, dDdy)
    x, y, z = ns[..., 0], ns[..., 1], ns[..., 2]
    rxz = np.maximum(x * x + z * z, 1e-30)
    us = np.arctan2(z, x) / (2 * math.pi) + 0.5
    vs = np.arccos(np.clip(y, -1.0, 1.0)) / math.pi
    gu = np.stack([-z / (2 * math.pi * rxz), np.zeros_like(x), x / (2 * math.pi * rxz)], -1)
    gv = np.stack([np.zeros_like(x), -1.0 / (math.pi * np.sqrt(np.maximum(1 - y * y, 1e-30))), np.zeros_like(x)], -1)
    sd = {
        "u": us, "v": vs,
        "dudx": np.sum(gu * dXdx, -1), "dvdx": np.sum(gv * dXdx, -1),
        "dudy": np.sum(gu * dXdy, -1), "dvdy": np.sum(gv * dXdy, -1),
    }
    # ground
    npl = np.broadcast_to(np.array([0.0, 1.0, 0.0]), D.shape)
    dPx, dPy = _differentials(np.where(use_p, tp, 1.0), D, npl, dDdx, dDdy)
    pdict = {
        "u": Xp[..., 0] / 4.0, "v": Xp[..., 2] / 4.0,
        "dudx": dPx[..., 0] / 4.0, "dvdx": dPx[..., 2] / 4.0,
        "dudy": dPy[..., 0] / 4.0, "dvdy": dPy[..., 2] / 4.0,
    }
    for k in ("u", "v", "dudx", "dvdx", "dudy", "dvdy"):
        g[k] = np.where(use_s, sd[k], np.where(use_p, pdict[k], g[k]))
    for i, k in enumerate(("nx", "ny", "nz")):
        g[k] = np.where(use_s, ns[..., i], np.where(use_p, npl[..., i], g[k]))
    for i, k in enumerate(("wx", "wy", "wz")):
        g[k] = np.where(use_s | use_p, wi[..., i], g[k])
    g["material_id"] = np.where(use_s | use_p, 0, -1).astype(np.int32)
    return g


def footprint_of(g):
    """Geometric (P, r, phi) of each pixel, FP64 (used only to redraw r)."""
    a = g["dudx"] ** 2 + g["dudy"] ** 2
    b = g["dudx"] * g["dvdx"] + g["dudy"] * g["dvdy"]
    c = g["dvdx"] ** 2 + g["dvdy"] ** 2
    P = np.abs(g["dudx"] * g["dvdy"] - g["dudy"] * g["dvdx"])
    s0 = 0.5 * (a + c) + np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.maximum(s0 / P, 1.0)
    phi = 0.5 * np.arctan2(2 * b, a - c)
    phi = np.where(phi < 0, phi + math.pi, phi)
    return P, r, phi


def redraw_ratio(g, r_new):
    """Keep P and phi, set the anisotropy ratio: J' = R(phi) diag(sqrt(Pr), sqrt(P/r))."""
    P, _, phi = footprint_of(g)
    live = g["material_id"] >= 0
    P = np.where(live & (P > 0), P, 1e-6)
    s0, s1 = np.sqrt(P * r_new), np.sqrt(P / r_new)
    cp, sp = np.cos(phi), np.sin(phi)
    g["dudx"] = np.where(live, cp * s0, g["dudx"])
    g["dvdx"] = np.where(live, sp * s0, g["dvdx"])
    g["dudy"] = np.where(live, -sp * s1, g["dudy"])
    g["dvdy"] = np.where(live, cp * s1, g["dvdy"])
    return g


def _light_dir(el, az, up_axis):
    ce, se = math.cos(el), math.sin(el)
    if up_axis == "z":
        return (ce * math.cos(az), ce * math.sin(az), se)
    return (ce * math.cos(az), se, ce * math.sin(az))


# ----------------------------------------------------------------------------------------
# Benchmark configurations
# ----------------------------------------------------------------------------------------
def view_plane_gbuffer(W, H, elevation_deg, fov_deg=40.0, height=1.0, uv_scale=1.0):
    """Unbounded plane z=0 with uv = uv_scale (x, y), seen from height `height`
    along a direction `elevation_deg` below the horizon (90: straight down).
    Pixels above the horizon miss (material -1)."""
    e = math.radians(elevation_deg)
    f = (0.0, math.cos(e), -math.sin(e))
    up = (0.0, math.sin(e), math.cos(e))
    eye = (0.0, 0.0, height)
    E, D, dDdx, dDdy = _camera(eye, tuple(np.add(eye, f)), up, fov_deg, W, H)
    n = np.array([0.0, 0.0, 1.0])
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -E[2] / D[..., 2]
    hit = (D[..., 2] < -1e-9) & (t > 0)
    t = np.where(hit, t, 1.0)
    X = E + t[..., None] * D
    g = _empty(H, W)
    nn = np.broadcast_to(n, D.shape)
    dXdx, dXdy = _differentials(t, D, nn, dDdx, dDdy)
    wi = -_normalize(D)
    g["u"] = np.where(hit, uv_scale * X[..., 0], 0.0)
    g["v"] = np.where(hit, uv_scale * X[..., 1], 0.0)
    g["dudx"] = np.where(hit, uv_scale * dXdx[..., 0], 1.0)
    g["dvdx"] = np.where(hit, uv_scale * dXdx[..., 1], 0.0)
    g["dudy"] = np.where(hit, uv_scale * dXdy[..., 0], 0.0)
    g["dvdy"] = np.where(hit, uv_scale * dXdy[..., 1], 1.0)
    g["nx"][:] = 0.0; g["ny"][:] = 0.0; g["nz"][:] = 1.0
    g["wx"], g["wy"], g["wz"] = wi[..., 0], wi[..., 1], wi[..., 2]
    g["material_id"] = np.where(hit, 0, -1).astype(np.int32)
    return g


PAPER_VIEWS = ("plane90", "plane25", "scattered")


def paper_setting(W=1920, H=1080, view="plane90", log10_density=5.0, seed=0):
    """The performance setting of the paper's Table 1 on synthetic inputs: one
    Beckmann material with alpha = 1.0 at a given flake density, one
    directional light, 1080p.  Views: a plane seen straight down (plane90), at
    25 degrees (plane25: footprints stretch towards the horizon, clustered
    anisotropy and split probes), and the plane90 footprints with the ratio
    redrawn per pixel, r ~ LogU[1, 64] (scattered anisotropy)."""
    if view not in PAPER_VIEWS:
        raise ValueError(f"view must be one of {PAPER_VIEWS}")
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    g = view_plane_gbuffer(W, H, 25.0 if view == "plane25" else 90.0)
    if view == "scattered":
        g = redraw_ratio(g, np.exp(rng.uniform(0.0, math.log(64.0), (H, W))))
    el = math.radians(rng.uniform(30, 70)); az = rng.uniform(0, 2 * math.pi)
    lights = [dict(dir=_light_dir(el, az, "z"), radiance=(1.0, 1.0, 1.0))]
    mats = [dict(ndf=1, alpha=1.0, R=DEFAULT_R, log10_density=float(log10_density),
                 micro_roughness=DEFAULT_MICRO, F0=DEFAULT_F0, seed=seed)]
    return _finish(g), mats, lights


def plain_forward(W=256, H=256, tilt_deg=60.0, seed=0):
    """Plane under a tilted camera, GGX alpha 0.3, 1e5 flakes per unit UV area,
    one directional light (elevation U(30,70) deg, azimuth U(0,360) deg)."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    g = plane_gbuffer(W, H, tilt_deg)
    el = math.radians(rng.uniform(30, 70)); az = rng.uniform(0, 2 * math.pi)
    lights = [dict(dir=_light_dir(el, az, "z"), radiance=(1.0, 1.0, 1.0))]
    mats = [dict(ndf=0, alpha=0.3, R=DEFAULT_R, log10_density=5.0, micro_roughness=DEFAULT_MICRO,
                 F0=DEFAULT_F0, seed=seed)]
    return _finish(g), mats, lights


def sphere_forward(W=1920, H=1080, seed=1, redraw=True):
    """Sphere + ground plane, r ~ LogU[1,16] per pixel (redraw=True, scattered
    anisotropy) or the geometric footprint (redraw=False, clustered anisotropy),
    per-pixel alpha ~ U(0.05,0.5) and log10 N ~ U(3,7), one light."""
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    g = sphere_gbuffer(W, H, rng)
    if redraw:
        g = redraw_ratio(g, np.exp(rng.uniform(0.0, math.log(16.0), (H, W))))
    g["alpha_px"] = rng.uniform(0.05, 0.5, (H, W))
    g["log10_density_px"] = rng.uniform(3.0, 7.0, (H, W))
    el = math.radians(rng.uniform(20, 70)); az = rng.uniform(0, 2 * math.pi)
    lights = [dict(dir=_light_dir(el, az, "y"), radiance=(1.0, 1.0, 1.0))]
    mats = [dict(ndf=0, alpha=0.3, R=DEFAULT_R, log10_density=5.0, micro_roughness=DEFAULT_MICRO,
                 F0=DEFAULT_F0, seed=seed)]
    return _finish(g), mats, lights


def four_k(W=3840, H=2160, seed=3, n_mat=8, n_light=4, tile=16, grazing_frac=0.3,
           n_probe_max=21, k_max=4):
    """Sphere + ground plane; 8 GGX materials (alpha ~ U(0.02,0.6), log10 N ~
    U(3,8), seeds 0-7) assigned by a Voronoi map over 64 seeded sites; 4 lights
    (elevation U(20,80) deg, seeded colours).  Footprints are redrawn per 16x16
    tile: 70% in range (r ~ LogU[1,16]) and 30% grazing (n_pr ~ LogU-int[2,21],
    r = 16 n_pr U(0.9,1]).  Tiles in the left half are clustered (one draw per
    tile); pixels in the right half draw independently (scattered)."""
    rng = np.random.Generator(np.random.PCG64(3000 + seed))
    # materials, lights and the material map come from their own stream so that
    # they do not depend on the frame size
    rng_m = np.random.Generator(np.random.PCG64(3100 + seed))
    mats = [dict(ndf=0, alpha=float(rng_m.uniform(0.02, 0.6)), R=DEFAULT_R,
                 log10_density=float(rng_m.uniform(3.0, 8.0)), micro_roughness=DEFAULT_MICRO,
                 F0=DEFAULT_F0, seed=m) for m in range(n_mat)]
    lights = []
    for _ in range(n_light):
        el = math.radians(rng_m.uniform(20, 80)); az = rng_m.uniform(0, 2 * math.pi)
        col = tuple(float(c) for c in rng_m.uniform(0.3, 1.0, 3))
        lights.append(dict(dir=_light_dir(el, az, "y"), radiance=col))
    sites = rng_m.uniform(0, 1, (64, 2)) * np.array([W, H])
    labels = rng_m.integers(0, n_mat, 64)
    g = sphere_gbuffer(W, H, rng)
    rmax = float(2 ** k_max)
    ty, tx = (H + tile - 1) // tile, (W + tile - 1) // tile

    def draw(shape):
        graz = rng.uniform(0, 1, shape) < grazing_frac
        r_in = np.exp(rng.uniform(0.0, math.log(rmax), shape))
        npr = np.floor(np.exp(rng.uniform(math.log(2.0), math.log(n_probe_max + 1.0), shape)))
        npr = np.clip(npr, 2, n_probe_max)
        r_gr = rmax * npr * (1.0 - 0.1 * rng.uniform(0, 1, shape))
        return np.where(graz, r_gr, r_in)

    r_tile = np.repeat(np.repeat(draw((ty, tx)), tile, 0), tile, 1)[:H, :W]
    r_pix = draw((H, W))
    left = (np.arange(W) < W // 2)[None, :]
    g = redraw_ratio(g, np.where(left, r_tile, r_pix))
    from scipy.spatial import cKDTree
    yy, xx = np.mgrid[0:H, 0:W]
    _, site = cKDTree(sites).query(np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5], -1))
    mat_map = labels[site.reshape(H, W)].astype(np.int32)
    g["material_id"] = np.where(g["material_id"] >= 0, mat_map, -1).astype(np.int32)
    return _finish(g), mats, lights


def batched_views(n_views=64, seed=4, side_min=128, side_max=2048, max_side=None, workers=8):
    """n_views square views, side ~ round(exp U(ln 128, ln 2048)), each a
    sphere_forward scene from its own random camera (seed 100 + view index,
    so the views do not depend on the order they are built in; `workers`
    threads build them)."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.Generator(np.random.PCG64(4000 + seed))
    sides = np.round(np.exp(rng.uniform(math.log(side_min), math.log(side_max), n_views))).astype(int)
    if max_side is not None:
        sides = np.minimum(sides, max_side)
    # largest views first, so that the pool's last tasks are short
    order = sorted(range(n_views), key=lambda i: -int(sides[i]))
    with ThreadPoolExecutor(max_workers=max(1, int(workers))) as ex:
        built = dict(zip(order, ex.map(lambda i: sphere_forward(int(sides[i]), int(sides[i]), seed=100 + i), order)))
    views = [built[i][0] for i in range(n_views)]
    mats, lights = built[0][1], built[0][2]
    return views, mats, lights


def backward_scene(W=1024, H=1024, seed=5):
    """Sphere + ground, r ~ LogU[1,16], one global GGX material (alpha 0.3,
    N = 1e5), one light d0.  Also returns the perturbed target parameters:
    alpha + 0.03, ln N + 0.3, d0 rotated 3 deg about a seeded axis."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    g = sphere_gbuffer(W, H, rng)
    g = redraw_ratio(g, np.exp(rng.uniform(0.0, math.log(16.0), (H, W))))
    el = math.radians(rng.uniform(30, 60)); az = rng.uniform(0, 2 * math.pi)
    d0 = np.array(_light_dir(el, az, "y"))
    mats = [dict(ndf=0, alpha=0.3, R=DEFAULT_R, log10_density=5.0, micro_roughness=DEFAULT_MICRO,
                 F0=DEFAULT_F0, seed=seed)]
    lights = [dict(dir=tuple(d0), radiance=(1.0, 1.0, 1.0))]
    axis = _normalize(rng.normal(size=3))
    ang = math.radians(3.0)
    d1 = (d0 * math.cos(ang) + np.cross(axis, d0) * math.sin(ang)
          + axis * np.dot(axis, d0) * (1 - math.cos(ang)))
    tmats = [dict(mats[0], alpha=0.33, log10_density=5.0 + 0.3 / math.log(10.0))]
    tlights = [dict(dir=tuple(d1), radiance=(1.0, 1.0, 1.0))]
    return _finish(g), mats, lights, tmats, tlights


def ragged_plane(W, H, seed=0, n_mat=3, n_light=2):
    """Small odd-sized plane with several materials, a skipped region and a few
    invalid pixels -- edge cases for parity tests."""
    rng = np.random.Generator(np.random.PCG64(6000 + seed))
    g = plane_gbuffer(W, H, 55.0)
    mid = rng.integers(0, n_mat, (H, W)).astype(np.int32)
    g["material_id"] = np.where(g["material_id"] >= 0, mid, -1).astype(np.int32)
    mats = [dict(ndf=m % 2, alpha=float(rng.uniform(0.1, 0.6)), R=DEFAULT_R,
                 log10_density=float(rng.uniform(4, 7)), micro_roughness=DEFAULT_MICRO,
                 F0=float(rng.uniform(0.04, 1.0)), seed=int(rng.integers(0, 2**32)))
            for m in range(n_mat)]
    lights = [dict(dir=_light_dir(math.radians(rng.uniform(25, 75)), rng.uniform(0, 2 * math.pi), "z"),
                   radiance=tuple(float(c) for c in rng.uniform(0.2, 1.0, 3))) for _ in range(n_light)]
    out = _finish(g)
    return out, mats, lights
