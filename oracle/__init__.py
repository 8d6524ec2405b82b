"""FP64 CPU oracle for per-pixel glint shading -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2306_05051_amd``) never imports it, and it imports nothing from
the product: the two implementations share no code.  See the header of
``glint_oracle.c`` for the step-by-step correspondence with the paper.

Inputs are the same FP32 G-buffer planes the GPU reads, given as a dict of
numpy arrays of shape (H, W): u, v, dudx, dvdx, dudy, dvdy, nx, ny, nz,
wx, wy, wz, optional material_id (int32), alpha_px, log10_density_px and
tangent planes tx, ty, tz (all three or none).
Materials are dicts with keys ndf, alpha, R, log10_density,
micro_roughness, F0, seed; lights are dicts with keys dir, radiance.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glint_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PLANES = ("u", "v", "dudx", "dvdx", "dudy", "dvdy", "nx", "ny", "nz", "wx", "wy", "wz")

FLAG_SHADED, FLAG_CLAMP_RATIO, FLAG_CLAMP_P, FLAG_BAD_INPUT = 1, 2, 4, 8
FLAG_BACKFACING, FLAG_SKIPPED, FLAG_BAD_MAT = 16, 32, 64
MARGIN_KINDS = ("none", "nprobe", "ratio", "orient", "triangle", "tetra", "lattice",
                "angular", "gate", "count", "light", "view", "zk_switch", "pclamp", "tangent")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict FP64: no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _GBuf(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("stride", C.c_int64)] + \
               [(n, C.c_void_p) for n in PLANES] + \
               [("material_id", C.c_void_p), ("alpha_px", C.c_void_p), ("log10_density_px", C.c_void_p),
                ("tx", C.c_void_p), ("ty", C.c_void_p), ("tz", C.c_void_p)]


class _Mat(C.Structure):
    _fields_ = [("ndf", C.c_int32), ("alpha", C.c_float), ("R", C.c_float),
                ("log10_density", C.c_float), ("micro_roughness", C.c_float),
                ("F0", C.c_float), ("seed", C.c_uint32)]


class _Light(C.Structure):
    _fields_ = [("dir", C.c_float * 3), ("radiance", C.c_float * 3)]


class _Params(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("n_probe_max", C.c_int32), ("rounding", C.c_int32),
                ("rng_log2", C.c_int32), ("rng_seed", C.c_uint32), ("count_law", C.c_int32)]


_DBG_FIELDS = [("flags", np.uint32), ("n_probe", np.int32), ("level", np.int32),
               ("cell", np.uint32), ("key_sum", np.uint32), ("akey_sum", np.uint32),
               ("theta_sum", np.uint32), ("count_sum", np.uint32), ("n_open", np.uint32),
               ("n_gate", np.uint32), ("n_live", np.uint32), ("margin", np.float64),
               ("margin_kind", np.int32), ("margin_pos", np.float64), ("margin_pos_kind", np.int32)]


class _Dbg(C.Structure):
    _fields_ = ([(n, C.c_void_p) for n, _ in _DBG_FIELDS] + [("b_light", C.c_void_p), ("lit", C.c_void_p)]
                + [("dump_slot", C.c_void_p), ("dump_capacity", C.c_int32), ("dump_probes", C.c_int32),
                   ("dump_key", C.c_void_p), ("dump_beta", C.c_void_p), ("dump_theta", C.c_void_p),
                   ("dump_count", C.c_void_p)])


class _Nodes(C.Structure):
    _fields_ = [("n", C.c_int), ("l", C.c_int * 4), ("k", C.c_int * 4), ("m", C.c_int * 4),
                ("w", C.c_double * 4), ("level", C.c_int), ("kappa", C.c_int), ("j", C.c_int),
                ("tri", C.c_int), ("pivot", C.c_int), ("D", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.og_shade.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), C.c_int, C.POINTER(_Light), C.c_int,
                               C.POINTER(_Params), C.c_void_p, C.POINTER(_Dbg), C.c_int, C.c_int, C.c_int]
        L.og_grad.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), C.c_int, C.POINTER(_Light), C.c_int,
                              C.POINTER(_Params), C.c_void_p, C.c_double, C.c_int, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.og_grad_dual.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), C.c_int, C.POINTER(_Light), C.c_int,
                                   C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int]
        L.og_fmix32.argtypes = [C.c_uint32]
        L.og_fmix32.restype = C.c_uint32
        L.og_hash_step.argtypes = [C.c_uint32, C.c_uint32]
        L.og_hash_step.restype = C.c_uint32
        L.og_rng_table_entry.argtypes = [C.c_uint32, C.c_uint32]
        L.og_rng_table_entry.restype = C.c_uint32
        L.og_texel_hash.argtypes = [C.c_uint32] + [C.c_int] * 8
        L.og_texel_hash.restype = C.c_uint32
        L.og_ndtri.argtypes = [C.c_double]
        L.og_ndtri.restype = C.c_double
        L.og_ndf.argtypes = [C.c_int, C.c_double, C.c_double]
        L.og_ndf.restype = C.c_double
        L.og_smith_lambda.argtypes = [C.c_int, C.c_double, C.c_double]
        L.og_smith_lambda.restype = C.c_double
        L.og_footprint.argtypes = [C.c_double] * 4 + [C.POINTER(C.c_double)] * 4
        L.og_grid_nodes.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.POINTER(_Nodes),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.og_simplex.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                 C.c_int * 3, C.c_int * 3, C.c_double * 3,
                                 C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.og_gated_count.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]
        L.og_gated_count.restype = C.c_double
        L.og_onb.argtypes = [C.c_double * 3, C.c_double * 3, C.c_double * 3]
        L.og_tangent_frame.argtypes = [C.c_double * 3] * 4
        L.og_tangent_frame.restype = C.c_int
        L.og_angular_texels.argtypes = [C.c_double * 3, C.c_double * 3, C.c_double * 3, C.c_double,
                                        C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_double * 4]
        L.og_probe_centre.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int, C.POINTER(C.c_double),
                                                         C.POINTER(C.c_double)]
        L.og_zk_count.argtypes = [C.c_double, C.c_double, C.c_uint32, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.og_zk_count.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _gbuf(gb):
    H, W = gb["u"].shape
    keep = {}
    s = _GBuf()
    s.width, s.height, s.stride = W, H, W
    for n in PLANES:
        a = np.ascontiguousarray(gb[n], dtype=np.float32)
        keep[n] = a
        setattr(s, n, a.ctypes.data)
    for n, dt in (("material_id", np.int32), ("alpha_px", np.float32), ("log10_density_px", np.float32),
                  ("tx", np.float32), ("ty", np.float32), ("tz", np.float32)):
        if gb.get(n) is not None:
            a = np.ascontiguousarray(gb[n], dtype=dt)
            keep[n] = a
            setattr(s, n, a.ctypes.data)
        else:
            setattr(s, n, None)
    return s, keep, H, W


def _mats(materials):
    arr = (_Mat * len(materials))()
    for i, m in enumerate(materials):
        arr[i] = _Mat(int(m.get("ndf", 0)), float(m["alpha"]), float(m.get("R", 0.034)),
                      float(m["log10_density"]), float(m.get("micro_roughness", 0.02)),
                      float(m.get("F0", 1.0)), int(m.get("seed", 0)) & 0xFFFFFFFF)
    return arr


def _lights(lights):
    arr = (_Light * max(1, len(lights)))()
    for i, l in enumerate(lights):
        arr[i].dir[:] = [float(x) for x in l["dir"]]
        arr[i].radiance[:] = [float(x) for x in l.get("radiance", (1.0, 1.0, 1.0))]
    return arr


def shade(gb, materials, lights, k_max=4, n_probe_max=21, rounding=0, debug=False,
          rows=None, n_threads=0, rng_table=None, count_law=0, dump_pixels=None, dump_probes=4):
    """FP64 radiance [3, H, W]; with debug=True also a dict of per-pixel planes.

    rng_table=None hashes every gate uniform from its keys; rng_table=(log2,
    seed) reads them from the table of 2**log2 words whose entry i is
    hash_step(seed, i) (log2 in 1..32), at the index (texel key XOR angular
    key) mod 2**log2.

    count_law=1 counts with the Zirr-Kaplanyan baseline (zk_count per texel,
    outputs mixed with the node weights); its debug planes then hold: n_open
    the counts on the Gaussian branch, n_live the Bernoulli trials drawn,
    count_sum the sum of the integer counts, lit the lights with a count > 0.

    dump_pixels: (y, x) pixels whose texel-level decisions are dumped (with
    debug=True): planes["dump"] then holds, per listed pixel and probe
    k < dump_probes, "key" and "beta" [n, dump_probes, 4, 3] (texel key and
    barycentric weight of node g, vertex e) and "theta" and "count"
    [n, dump_probes, n_light, 4, 3, 4] (slot-0 word and count of angular
    texel a), zero where there is no texel."""
    L = lib()
    s, keep, H, W = _gbuf(gb)
    mats, lts = _mats(materials), _lights(lights)
    log2, seed = (0, 0) if rng_table is None else (int(rng_table[0]), int(rng_table[1]) & 0xFFFFFFFF)
    if rng_table is not None and not 1 <= log2 <= 32:
        raise ValueError("rng_table log2 must be in 1..32")
    prm = _Params(k_max, n_probe_max, rounding, log2, seed, count_law)
    out = np.zeros((3, H, W), np.float64)
    dbg = None
    planes = {}
    if debug:
        dbg = _Dbg()
        for n, dt in _DBG_FIELDS:
            planes[n] = np.zeros((H, W), dt)
            setattr(dbg, n, planes[n].ctypes.data)
        planes["b_light"] = np.zeros((max(1, len(lights)), H, W), np.float64)
        dbg.b_light = planes["b_light"].ctypes.data
        planes["lit"] = np.zeros((H, W), np.uint32)
        dbg.lit = planes["lit"].ctypes.data
        if dump_pixels is not None and len(dump_pixels):
            yx = np.asarray(dump_pixels, np.int64).reshape(-1, 2)
            slot = np.full((H, W), -1, np.int32)
            slot[yx[:, 0], yx[:, 1]] = np.arange(len(yx), dtype=np.int32)
            n, P, NL = len(yx), int(dump_probes), len(lights)
            dump = {"slot": slot, "key": np.zeros((n, P, 4, 3), np.uint32),
                    "beta": np.zeros((n, P, 4, 3), np.float64),
                    "theta": np.zeros((n, P, NL, 4, 3, 4), np.uint32),
                    "count": np.zeros((n, P, NL, 4, 3, 4), np.float64)}
            dbg.dump_slot = slot.ctypes.data
            dbg.dump_capacity, dbg.dump_probes = n, P
            for k in ("key", "beta", "theta", "count"):
                setattr(dbg, "dump_" + k, dump[k].ctypes.data)
            planes["dump"] = dump
    elif dump_pixels is not None:
        raise ValueError("dump_pixels needs debug=True")
    r0, r1 = (0, H) if rows is None else rows
    rc = L.og_shade(C.byref(s), mats, len(materials), lts, len(lights), C.byref(prm),
                    out.ctypes.data, C.byref(dbg) if dbg is not None else None, r0, r1, n_threads)
    if rc != 0:
        raise ValueError(f"og_shade failed ({rc})")
    del keep
    return (out, planes) if debug else out


def grad(gb, materials, lights, grad_out, step=1e-6, frozen=True, k_max=4, n_probe_max=21,
         n_threads=0):
    """Gradient of sum(grad_out * L) (relaxed counts) w.r.t. each material's alpha
    and ln N and each light's raw direction.  Returns (g_alpha, g_lnN, g_dir, flip)."""
    L = lib()
    s, keep, H, W = _gbuf(gb)
    mats, lts = _mats(materials), _lights(lights)
    prm = _Params(k_max, n_probe_max, 1, 0, 0)
    go = np.ascontiguousarray(grad_out, dtype=np.float64).reshape(3, H, W)
    ga = np.zeros(len(materials)); gn = np.zeros(len(materials)); gd = np.zeros(3 * len(lights))
    flip = np.zeros((H, W), np.uint8)
    rc = L.og_grad(C.byref(s), mats, len(materials), lts, len(lights), C.byref(prm), go.ctypes.data,
                   float(step), int(bool(frozen)), ga.ctypes.data, gn.ctypes.data, gd.ctypes.data,
                   flip.ctypes.data, n_threads)
    if rc != 0:
        raise ValueError(f"og_grad failed ({rc})")
    del keep
    return ga, gn, gd.reshape(len(lights), 3), flip


def grad_dual(gb, materials, lights, grad_out, k_max=4, n_probe_max=21, n_threads=0):
    """The same gradient as grad(frozen=True) by forward-mode derivatives (dual
    numbers carried through the relaxed forward, decisions taken on the
    values).  Returns (g_alpha, g_lnN, g_dir, loss) with loss = sum(grad_out * L)."""
    L = lib()
    s, keep, H, W = _gbuf(gb)
    mats, lts = _mats(materials), _lights(lights)
    prm = _Params(k_max, n_probe_max, 1, 0, 0)
    go = np.ascontiguousarray(grad_out, dtype=np.float64).reshape(3, H, W)
    ga = np.zeros(len(materials)); gn = np.zeros(len(materials)); gd = np.zeros(3 * len(lights))
    loss = np.zeros(1)
    rc = L.og_grad_dual(C.byref(s), mats, len(materials), lts, len(lights), C.byref(prm), go.ctypes.data,
                        ga.ctypes.data, gn.ctypes.data, gd.ctypes.data, loss.ctypes.data, n_threads)
    if rc != 0:
        raise ValueError(f"og_grad_dual failed ({rc})")
    del keep
    return ga, gn, gd.reshape(len(lights), 3), float(loss[0])


# ---- scalar entry points used by the pin tests ------------------------------------------
def fmix32(h):
    return lib().og_fmix32(h & 0xFFFFFFFF)


def hash_step(h, w):
    return lib().og_hash_step(h & 0xFFFFFFFF, w & 0xFFFFFFFF)


def rng_table_entry(seed, i):
    """Entry i of the random-number table of the given seed: hash_step(seed, i)."""
    return lib().og_rng_table_entry(seed & 0xFFFFFFFF, i & 0xFFFFFFFF)


def texel_hash(seed, l, k, m, i, j, ai, aj, s):
    """32-bit hash of the full key of one per-texel random number."""
    return lib().og_texel_hash(seed & 0xFFFFFFFF, l, k, m, i, j, ai, aj, s)


def uniform(bits):
    """The uniform in (0,1) a hash output stands for: (2 (h >> 9) + 1) 2^-24."""
    return (2.0 * (bits >> 9) + 1.0) * 2.0**-24


def ndtri(q):
    return lib().og_ndtri(float(q))


def ndf(kind, alpha, cos_m):
    return lib().og_ndf(int(kind), float(alpha), float(cos_m))


def smith_lambda(kind, alpha, c):
    return lib().og_smith_lambda(int(kind), float(alpha), float(c))


def footprint(dudx, dvdx, dudy, dvdy):
    """(P, r, phi, sigma0) or None for a degenerate Jacobian."""
    P, r, phi, s0 = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    ok = lib().og_footprint(float(dudx), float(dvdx), float(dudy), float(dvdy),
                            C.byref(P), C.byref(r), C.byref(phi), C.byref(s0))
    return (P.value, r.value, phi.value, s0.value) if ok else None


def grid_nodes(Pk, rk, phi, k_max=4):
    """Tetrahedron vertices of the (area, ratio, orientation) grid family:
    list of (l, k, m, w) plus the cell description and the smallest margin."""
    n = _Nodes()
    mg, mk = (C.c_double * 2)(np.inf, np.inf), (C.c_int * 2)(0, 0)
    lib().og_grid_nodes(float(Pk), float(rk), float(phi), int(k_max), C.byref(n), mg, mk)
    nodes = [(n.l[i], n.k[i], n.m[i], n.w[i]) for i in range(n.n)]
    cell = dict(level=n.level, kappa=n.kappa, j=n.j, tri=n.tri, pivot=n.pivot, D=n.D)
    return nodes, cell, mg[0]


def simplex(cx, cy, l, k, m):
    vi, vj, beta = (C.c_int * 3)(), (C.c_int * 3)(), (C.c_double * 3)()
    mg, mk = (C.c_double * 2)(np.inf, np.inf), (C.c_int * 2)(0, 0)
    lib().og_simplex(float(cx), float(cy), int(l), int(k), int(m), vi, vj, beta, mg, mk)
    return list(zip(vi, vj)), list(beta), mg[0]


def gated_count(n, p, theta0, theta1, rounding=0):
    return lib().og_gated_count(float(n), float(p), float(theta0), float(theta1), int(rounding))


def zk_count(n, p, h0):
    """One count of the Zirr-Kaplanyan baseline from n trials, probability p and
    the texel's slot-0 word h0: (count, gaussian branch taken, trials drawn)."""
    g, t = C.c_int(), C.c_int()
    c = lib().og_zk_count(float(n), float(p), h0 & 0xFFFFFFFF, C.byref(g), C.byref(t))
    return c, g.value, t.value


def tangent_frame(n):
    """(t, b) of the unit normal n: the frame whose axes index the angular grid."""
    t, b = (C.c_double * 3)(), (C.c_double * 3)()
    lib().og_onb((C.c_double * 3)(*[float(x) for x in n]), t, b)
    return list(t), list(b)


def frame_of_tangent(n, t):
    """(t, b) of the unit normal n and a supplied tangent t (made orthogonal to
    n, b = n x t), or None when t is (nearly) parallel to n."""
    to, bo = (C.c_double * 3)(), (C.c_double * 3)()
    ok = lib().og_tangent_frame((C.c_double * 3)(*[float(x) for x in n]),
                                (C.c_double * 3)(*[float(x) for x in t]), to, bo)
    return (list(to), list(bo)) if ok else None


def angular_texels(h, t, b, micro):
    """Lower-left angular texel (ai, aj) of the half vector h in the frame
    (t, b) with cells of size micro, and the bilinear weights v[a] of texels
    (ai + (a & 1), aj + (a >> 1)) (Eq. 14)."""
    ai, aj, v = C.c_int(), C.c_int(), (C.c_double * 4)()
    d3 = lambda x: (C.c_double * 3)(*[float(c) for c in x])
    lib().og_angular_texels(d3(h), d3(t), d3(b), float(micro), C.byref(ai), C.byref(aj), v)
    return ai.value, aj.value, list(v)


def probe_centre(u, v, phi, sigma0, n_pr, kp):
    """Centre of sub-footprint kp of n_pr along the footprint's major axis."""
    cx, cy = C.c_double(), C.c_double()
    lib().og_probe_centre(float(u), float(v), float(phi), float(sigma0), int(n_pr), int(kp),
                          C.byref(cx), C.byref(cy))
    return cx.value, cy.value
