"""Thin Python binding of libglint.so (the C ABI declared in include/glint.h).

Argument marshalling only: every step of glint shading runs in the HIP
kernels.  PyTorch provides device memory and the current HIP stream.  The
binding refuses to run when the library is missing; there is no CPU path.

A G-buffer is a dict of CUDA tensors of shape (H, W), dtype float32
(u, v, dudx, dvdx, dudy, dvdy, nx, ny, nz, wx, wy, wz), an optional int32
``material_id``, optional float32 ``alpha_px`` / ``log10_density_px`` and
optional float32 tangent planes ``tx``, ``ty``, ``tz`` (all three or none).
Planes may be row-padded views (element stride 1 along a row, one common row
stride >= W for every plane, as ``to_device(..., stride=S)`` makes): the C
ABI's ``stride``.  Outputs then come back as views of the same row stride.
Materials are dicts (ndf, alpha, R, log10_density, micro_roughness, F0,
seed) and lights are dicts (dir, radiance), as in ``include/glint.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglint.so")
PLANES = ("u", "v", "dudx", "dvdx", "dudy", "dvdy", "nx", "ny", "nz", "wx", "wy", "wz")

GLINT_OK, GLINT_EINVAL, GLINT_ENULL, GLINT_ESHAPE = 0, -1, -2, -3
GLINT_EHIP, GLINT_EUNSUPPORTED, GLINT_ENOMEM, GLINT_ELIMIT = -4, -5, -6, -7
GLINT_NOALLOC_WORKSPACE_BYTES = 2097152
GLINT_TILE_W, GLINT_TILE_H = 16, 4           # glint_shade's tile (one 64-lane wave)
GLINT_MAX_MATERIALS, GLINT_MAX_LIGHTS, GLINT_MAX_K, GLINT_MAX_PROBES = 32, 16, 4, 64
GLINT_RNG_TABLE_MIN_LOG2, GLINT_RNG_TABLE_MAX_LOG2, GLINT_RNG_LDS_MAX_LOG2 = 8, 32, 13
GLINT_RNG_CACHED, GLINT_RNG_LDS = 0, 1
GLINT_FLAG_ZK_COUNT = 1
LAW_DISTRIBUTED, LAW_ZK = 0, 1      # counting laws of glint_shade (count_law=)
MAX_MATERIALS, MAX_LIGHTS = 32, 16


class GlintError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().glint_status_string(status).decode()
        if status == GLINT_EHIP:
            msg += f" (hipError {lib().glint_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


class _GBuf(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("stride", C.c_int64)] + \
               [(n, C.c_void_p) for n in PLANES] + \
               [("material_id", C.c_void_p), ("alpha_px", C.c_void_p), ("log10_density_px", C.c_void_p),
                ("tx", C.c_void_p), ("ty", C.c_void_p), ("tz", C.c_void_p)]


class _Mat(C.Structure):
    _fields_ = [("ndf", C.c_int32), ("alpha", C.c_float), ("R", C.c_float), ("log10_density", C.c_float),
                ("micro_roughness", C.c_float), ("F0", C.c_float), ("seed", C.c_uint32)]


class _Light(C.Structure):
    _fields_ = [("dir", C.c_float * 3), ("radiance", C.c_float * 3)]


class _Params(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("n_probe_max", C.c_int32), ("rounding", C.c_int32),
                ("flags", C.c_uint32)]


DEBUG_FIELDS = (("flags", torch.int32), ("n_probe", torch.int32), ("level", torch.int32),
                ("cell", torch.int32), ("key_sum", torch.int32), ("akey_sum", torch.int32),
                ("theta_sum", torch.int32), ("count_sum", torch.int32), ("n_open", torch.int32),
                ("n_gate", torch.int32), ("n_live", torch.int32))
WORK_FIELDS = ("n_live_small", "n_lit", "n_live_lit")   # work counters of the instrumented kernel (after b_light)


class _Debug(C.Structure):
    _fields_ = ([(n, C.c_void_p) for n, _ in DEBUG_FIELDS] + [("b_light", C.c_void_p)]
                + [(n, C.c_void_p) for n in WORK_FIELDS]
                + [("dump_slot", C.c_void_p), ("dump_capacity", C.c_int32), ("dump_probes", C.c_int32),
                   ("dump_key", C.c_void_p), ("dump_beta", C.c_void_p), ("dump_theta", C.c_void_p),
                   ("dump_count", C.c_void_p)])


class _Tune(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib():
    """Load libglint.so (built by paper_2306_05051_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2306_05051_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.glint_shade.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), i32, C.POINTER(_Light), i32,
                                  C.POINTER(_Params), vp, C.POINTER(_Debug), vp, C.c_size_t, vp]
        L.glint_shade_noalloc.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), i32, C.POINTER(_Light), i32,
                                          C.POINTER(_Params), vp, vp]
        L.glint_rng_table_fill.argtypes = [vp, i32, C.c_uint32, vp]
        L.glint_shade_rng_table.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), i32, C.POINTER(_Light), i32,
                                            C.POINTER(_Params), vp, i32, i32, vp, C.POINTER(_Debug), vp,
                                            C.c_size_t, vp]
        L.glint_shade_workspace_bytes.argtypes = [i32, i32]
        L.glint_shade_workspace_bytes.restype = C.c_size_t
        L.glint_backward_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.glint_backward_workspace_bytes.restype = C.c_size_t
        L.glint_shade_backward.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), i32, C.POINTER(_Light), i32,
                                           C.POINTER(_Params), vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.glint_shade_lit.argtypes = [C.POINTER(_GBuf), C.POINTER(_Mat), i32, C.POINTER(_Light), i32,
                                      C.POINTER(_Params), vp, vp, vp, vp, C.c_size_t, vp]
        L.glint_plan_create.argtypes = [C.POINTER(_GBuf), C.POINTER(vp), i32, C.POINTER(_Mat), i32,
                                        C.POINTER(_Light), i32, C.POINTER(_Params), C.POINTER(_Tune),
                                        C.POINTER(vp)]
        L.glint_shade_batched.argtypes = [vp, i32, vp]
        L.glint_plan_destroy.argtypes = [vp]
        L.glint_plan_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32)]
        L.glint_texel_hash.argtypes = [vp, i64, vp, vp]
        L.glint_hash_step.argtypes = [vp, vp, i64, vp, vp]
        L.glint_ndtri.argtypes = [vp, i64, vp, vp]
        L.glint_status_string.argtypes = [C.c_int]
        L.glint_status_string.restype = C.c_char_p
        L.glint_last_hip_error.restype = C.c_int
        L.glint_version.restype = C.c_int
        _lib = L
    return _lib


def _check(status, where):
    if status != GLINT_OK:
        raise GlintError(status, where)


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor")
    return t.data_ptr()


TANGENT_PLANES = ("tx", "ty", "tz")


def row_stride(gb):
    """The common row stride (elements) of a G-buffer's planes."""
    return gb["u"].stride(0) if gb["u"].dim() == 2 and gb["u"].shape[0] > 1 else gb["u"].shape[-1]


def _plane_ptr(t, dtype, name, H, W, S):
    if not (t.is_cuda and t.dtype == dtype and tuple(t.shape) == (H, W)):
        raise ValueError(f"plane {name} must be a CUDA {dtype} tensor of shape {(H, W)}")
    if W > 0 and H > 0 and (t.stride(1) != 1 or (H > 1 and t.stride(0) != S)):
        raise ValueError(f"plane {name} must have element stride 1 and row stride {S}")
    return t.data_ptr()


def make_gbuffer(gb):
    """ctypes G-buffer descriptor for a dict of CUDA tensors of shape (H, W)
    sharing one row stride."""
    H, W = gb["u"].shape
    S = row_stride(gb)
    g = _GBuf()
    g.width, g.height, g.stride = W, H, S
    for n in PLANES:
        setattr(g, n, _plane_ptr(gb[n], torch.float32, n, H, W, S))
    g.material_id = _plane_ptr(gb["material_id"], torch.int32, "material_id", H, W, S) \
        if gb.get("material_id") is not None else None
    for n in ("alpha_px", "log10_density_px"):
        setattr(g, n, _plane_ptr(gb[n], torch.float32, n, H, W, S) if gb.get(n) is not None else None)
    have = [gb.get(n) is not None for n in TANGENT_PLANES]
    if any(have) and not all(have):
        raise ValueError("tangent planes tx, ty, tz: give all three or none")
    for n in TANGENT_PLANES:
        setattr(g, n, _plane_ptr(gb[n], torch.float32, n, H, W, S) if gb.get(n) is not None else None)
    return g


def _planes(n, H, W, S, dtype, device, fill=None):
    """n planes [n][H*S] as a tensor view of shape (n, H, W) (or (H, W) for n = 0)."""
    shape = (H, S) if n == 0 else (n, H, S)
    t = torch.empty(shape, dtype=dtype, device=device) if fill is None else \
        torch.full(shape, fill, dtype=dtype, device=device)
    return t[..., :W]


def _out_ptr(t, name, n, H, W, S, dtype=torch.float32):
    """pointer of an output of n planes [n][H*S] given as a (n, H, W) view (or (H, W) for n = 0)"""
    shape = (H, W) if n == 0 else (n, H, W)
    strides = (S, 1) if n == 0 else (H * S, S, 1)
    if not (t.is_cuda and t.dtype == dtype and tuple(t.shape) == shape):
        raise ValueError(f"{name} must be a CUDA {dtype} tensor of shape {shape}")
    if H * W > 0 and any(st != want for st, want, d in zip(t.stride(), strides, shape) if d > 1):
        raise ValueError(f"{name} must have strides {strides} (row stride {S})")
    return t.data_ptr()


def make_materials(materials):
    arr = (_Mat * max(1, len(materials)))()
    for i, m in enumerate(materials):
        arr[i] = _Mat(int(m.get("ndf", 0)), float(m["alpha"]), float(m.get("R", 0.034)),
                      float(m["log10_density"]), float(m.get("micro_roughness", 0.02)),
                      float(m.get("F0", 1.0)), int(m.get("seed", 0)) & 0xFFFFFFFF)
    return arr


def make_lights(lights):
    arr = (_Light * max(1, len(lights)))()
    for i, l in enumerate(lights):
        arr[i].dir[:] = [float(x) for x in l["dir"]]
        arr[i].radiance[:] = [float(x) for x in l.get("radiance", (1.0, 1.0, 1.0))]
    return arr


def make_params(k_max=4, n_probe_max=21, rounding=0, count_law=LAW_DISTRIBUTED):
    if count_law not in (LAW_DISTRIBUTED, LAW_ZK):
        raise ValueError("count_law must be LAW_DISTRIBUTED or LAW_ZK")
    return _Params(int(k_max), int(n_probe_max), int(rounding), GLINT_FLAG_ZK_COUNT if count_law == LAW_ZK else 0)


def to_device(gb_np, device="cuda", stride=None):
    """numpy G-buffer dict -> dict of CUDA tensors of shape (H, W); with
    stride = S > W each plane is a view of (H, S) storage (padded rows, the
    padding filled with NaN)."""
    out = {}
    for k, v in gb_np.items():
        if v is None:
            continue
        t = torch.from_numpy(v).to(device).contiguous()
        if stride is not None and stride != t.shape[1]:
            if stride < t.shape[1]:
                raise ValueError("stride must be at least the width")
            fill = -7 if t.dtype == torch.int32 else float("nan")
            pad = torch.full((t.shape[0], stride), fill, dtype=t.dtype, device=device)
            pad[:, :t.shape[1]] = t
            t = pad[:, :t.shape[1]]
        out[k] = t
    return out


def glint_shade_workspace_bytes(width, height):
    return lib().glint_shade_workspace_bytes(width, height)


def glint_shade(gbuf, materials, lights, k_max=4, n_probe_max=21, rounding=0, out=None, debug=False,
                workspace=None, stream=None, count_law=LAW_DISTRIBUTED, dump_pixels=None, dump_probes=4):
    """Radiance [3, H, W] float32 (and a dict of debug planes when debug=True).

    dump_pixels (with debug=True): (y, x) pixels whose texel-level decisions
    are dumped: planes["dump"] then holds, per listed pixel and probe
    k < dump_probes, "key" (int32) and "beta" [n, dump_probes, 4, 3] (texel key
    and barycentric weight of grid node g, lattice vertex e) and "theta"
    (int32) and "count" [n, dump_probes, n_light, 4, 3, 4] (slot-0 word and
    count of angular texel a), zero where there is no texel.

    workspace: None allocates the tile-order workspace (heaviest tiles first),
    False shades the tiles in row-major order without one, a uint8 CUDA tensor
    of at least glint_shade_workspace_bytes(W, H) bytes is used as given.
    count_law: LAW_DISTRIBUTED (the method) or LAW_ZK (the Zirr-Kaplanyan
    baseline, GLINT_FLAG_ZK_COUNT; rounding must be 0)."""
    return _shade(gbuf, materials, lights, k_max, n_probe_max, rounding, out, debug, workspace, stream, None,
                  count_law, dump_pixels, dump_probes)


def glint_shade_noalloc(gbuf, materials, lights, k_max=4, n_probe_max=21, rounding=0, out=None, stream=None,
                        count_law=LAW_DISTRIBUTED):
    """glint_shade (heaviest tiles first, same image) through the entry point
    that allocates nothing: its tile-order workspace is the library's static
    device array.  out: a float32 CUDA tensor [3, H, W] (allocated here when
    None, which the C call itself never does)."""
    g = make_gbuffer(gbuf)
    H, W = gbuf["u"].shape
    S = g.stride
    if out is None:
        out = _planes(3, H, W, S, torch.float32, gbuf["u"].device)
    st = lib().glint_shade_noalloc(C.byref(g), make_materials(materials), len(materials), make_lights(lights),
                                   len(lights), C.byref(make_params(k_max, n_probe_max, rounding, count_law)),
                                   _out_ptr(out, "out", 3, H, W, S), _stream(stream))
    _check(st, "glint_shade_noalloc")
    return out


RNG_CACHED, RNG_LDS = GLINT_RNG_CACHED, GLINT_RNG_LDS


def glint_rng_table_fill(log2_words, seed, table=None, stream=None):
    """Random-number table of 2**log2_words words (as int32), entry i = H(seed, i),
    filled on the GPU.  table: an int32 CUDA tensor of that many elements, or None."""
    n = 1 << int(log2_words)
    if table is None:
        table = torch.empty(n, dtype=torch.int32, device="cuda")
    elif table.numel() < n:
        raise ValueError("table is smaller than 2**log2_words words")
    _check(lib().glint_rng_table_fill(_dev_ptr(table, torch.int32, "table"), int(log2_words),
                                      int(seed) & 0xFFFFFFFF, _stream(stream)), "glint_rng_table_fill")
    return table


def glint_shade_rng_table(gbuf, materials, lights, table, log2_words, placement=RNG_CACHED, k_max=4,
                          n_probe_max=21, rounding=0, out=None, debug=False, workspace=None, stream=None):
    """glint_shade with the gate and count uniforms read from a random-number
    table (int32 CUDA tensor of at least 2**log2_words words) at index
    (texel key ^ angular key) mod 2**log2_words; placement RNG_CACHED reads it
    through the caches, RNG_LDS from a per-tile copy in LDS."""
    if table.numel() < (1 << int(log2_words)):
        raise ValueError("table is smaller than 2**log2_words words")
    rng = (_dev_ptr(table, torch.int32, "table"), int(log2_words), int(placement))
    return _shade(gbuf, materials, lights, k_max, n_probe_max, rounding, out, debug, workspace, stream, rng)


def _shade(gbuf, materials, lights, k_max, n_probe_max, rounding, out, debug, workspace, stream, rng,
           count_law=LAW_DISTRIBUTED, dump_pixels=None, dump_probes=4):
    L = lib()
    g = make_gbuffer(gbuf)
    H, W = gbuf["u"].shape
    S = g.stride
    dev = gbuf["u"].device
    if out is None:
        out = _planes(3, H, W, S, torch.float32, dev)
    out_ptr = _out_ptr(out, "out", 3, H, W, S)
    nbytes = L.glint_shade_workspace_bytes(W, H)
    if workspace is False or nbytes == 0:
        ws_ptr, ws_bytes = None, 0
    else:
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        ws_ptr, ws_bytes = _dev_ptr(workspace, torch.uint8, "workspace"), workspace.numel()
    dbg = None
    planes = {}
    if debug:
        dbg = _Debug()
        for n, dt in DEBUG_FIELDS:
            planes[n] = _planes(0, H, W, S, dt, dev, fill=0)
            setattr(dbg, n, planes[n].data_ptr())
        planes["b_light"] = _planes(max(1, len(lights)), H, W, S, torch.float32, dev, fill=0)
        dbg.b_light = planes["b_light"].data_ptr()
        for n in WORK_FIELDS:
            planes[n] = _planes(0, H, W, S, torch.int32, dev, fill=0)
            setattr(dbg, n, planes[n].data_ptr())
        if dump_pixels is not None and len(dump_pixels):
            yx = torch.as_tensor(dump_pixels, dtype=torch.int64).reshape(-1, 2)
            n, P, NL = yx.shape[0], int(dump_probes), len(lights)
            slot = _planes(0, H, W, S, torch.int32, dev, fill=-1)
            slot[yx[:, 0].to(dev), yx[:, 1].to(dev)] = torch.arange(n, dtype=torch.int32, device=dev)
            dump = {"slot": slot,
                    "key": torch.zeros((n, P, 4, 3), dtype=torch.int32, device=dev),
                    "beta": torch.zeros((n, P, 4, 3), dtype=torch.float32, device=dev),
                    "theta": torch.zeros((n, P, NL, 4, 3, 4), dtype=torch.int32, device=dev),
                    "count": torch.zeros((n, P, NL, 4, 3, 4), dtype=torch.float32, device=dev)}
            dbg.dump_slot = slot.data_ptr()
            dbg.dump_capacity, dbg.dump_probes = n, P
            for k in ("key", "beta", "theta", "count"):
                setattr(dbg, "dump_" + k, dump[k].data_ptr())
            planes["dump"] = dump
    elif dump_pixels is not None:
        raise ValueError("dump_pixels needs debug=True")
    prm = make_params(k_max, n_probe_max, rounding, count_law)
    if rng is None:
        st = glint_shade_raw(g, make_materials(materials), len(materials), make_lights(lights), len(lights),
                             prm, out_ptr, dbg, _stream(stream), ws_ptr, ws_bytes)
        _check(st, "glint_shade")
    else:
        st = L.glint_shade_rng_table(C.byref(g), make_materials(materials), len(materials), make_lights(lights),
                                     len(lights), C.byref(prm), rng[0], rng[1], rng[2], out_ptr,
                                     C.byref(dbg) if dbg is not None else None, ws_ptr, ws_bytes, _stream(stream))
        _check(st, "glint_shade_rng_table")
    return (out, planes) if debug else out


def glint_shade_raw(g, mats, n_mat, lts, n_light, prm, out_ptr, dbg, stream_ptr, ws_ptr=None, ws_bytes=0):
    return lib().glint_shade(C.byref(g), mats, n_mat, lts, n_light, C.byref(prm), out_ptr,
                             C.byref(dbg) if dbg is not None else None, ws_ptr, ws_bytes, stream_ptr)


def glint_backward_workspace_bytes(width, height, n_mat, n_light):
    return lib().glint_backward_workspace_bytes(width, height, n_mat, n_light)


def glint_shade_lit(gbuf, materials, lights, k_max=4, n_probe_max=21, rounding=1, out=None, lit=None,
                    probes=None, workspace=None, stream=None):
    """(radiance [3, H, W], lit [H, W] int16, probes [H, W] int32): glint_shade that
    also records, per pixel, the bit masks of the lights and of the probes with
    an open gate, for glint_shade_backward."""
    L = lib()
    g = make_gbuffer(gbuf)
    H, W = gbuf["u"].shape
    S = g.stride
    dev = gbuf["u"].device
    if out is None:
        out = _planes(3, H, W, S, torch.float32, dev)
    if lit is None:
        lit = _planes(0, H, W, S, torch.int16, dev)
    if probes is None:
        probes = _planes(0, H, W, S, torch.int32, dev)
    nbytes = L.glint_shade_workspace_bytes(W, H)
    if workspace is None or workspace is False:
        workspace = torch.empty(max(1, nbytes), dtype=torch.uint8, device=dev)
    st = L.glint_shade_lit(C.byref(g), make_materials(materials), len(materials), make_lights(lights),
                           len(lights), C.byref(make_params(k_max, n_probe_max, rounding)),
                           _out_ptr(out, "out", 3, H, W, S), _out_ptr(lit, "lit", 0, H, W, S, torch.int16),
                           _out_ptr(probes, "probes", 0, H, W, S, torch.int32),
                           _dev_ptr(workspace, torch.uint8, "workspace"), nbytes, _stream(stream))
    _check(st, "glint_shade_lit")
    return out, lit, probes


def glint_shade_backward(gbuf, materials, lights, grad_out, k_max=4, n_probe_max=21, workspace=None,
                         stream=None, lit=None, probes=None):
    """(grad_alpha[n_mat], grad_ln_density[n_mat], grad_light_dir[n_light, 3]) of
    sum(grad_out * L) for the relaxed forward.  lit, probes: the masks from
    glint_shade_lit on the same inputs (skip the pixels, lights and probes
    without an open gate; the same terms), or None to evaluate every gate."""
    L = lib()
    g = make_gbuffer(gbuf)
    H, W = gbuf["u"].shape
    S = g.stride
    dev = gbuf["u"].device
    nm, nl = len(materials), len(lights)
    if grad_out.shape != (3, H, W):
        raise ValueError(f"grad_out must have shape {(3, H, W)}")
    try:
        go_ptr = _out_ptr(grad_out, "grad_out", 3, H, W, S)
    except ValueError:           # repack into the G-buffer's row stride
        go = _planes(3, H, W, S, torch.float32, dev, fill=0.0)
        go.copy_(grad_out)
        grad_out = go
        go_ptr = _out_ptr(grad_out, "grad_out", 3, H, W, S)
    ga = torch.empty(nm, dtype=torch.float32, device=dev)
    gn = torch.empty(nm, dtype=torch.float32, device=dev)
    gd = torch.empty((nl, 3), dtype=torch.float32, device=dev)
    nbytes = L.glint_backward_workspace_bytes(W, H, nm, nl)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(1, nbytes), dtype=torch.uint8, device=dev)
    st = L.glint_shade_backward(C.byref(g), make_materials(materials), nm, make_lights(lights), nl,
                                C.byref(make_params(k_max, n_probe_max, 1)),
                                go_ptr,
                                None if lit is None else _out_ptr(lit, "lit", 0, H, W, S, torch.int16),
                                None if probes is None else _out_ptr(probes, "probes", 0, H, W, S, torch.int32),
                                ga.data_ptr(), gn.data_ptr(), gd.data_ptr(), workspace.data_ptr(),
                                nbytes, _stream(stream))
    _check(st, "glint_shade_backward")
    return ga, gn, gd


class GlintPlan:
    """Batched persistent shading of many views (glint_plan_create /
    glint_shade_batched / glint_plan_destroy)."""

    def __init__(self, gbufs, outs, materials, lights, k_max=4, n_probe_max=21, rounding=0, tune=None):
        L = lib()
        n = len(gbufs)
        self._gb = (_GBuf * n)(*[make_gbuffer(g) for g in gbufs])
        self._outs = (C.c_void_p * n)(*[_out_ptr(o, "out", 3, gb.height, gb.width, gb.stride)
                                        for o, gb in zip(outs, self._gb)])
        self._keep = (gbufs, outs)
        t = None
        if tune is not None:
            t = _Tune(int(tune[0]), int(tune[1]), int(tune[2]), 0)
        h = C.c_void_p()
        st = L.glint_plan_create(self._gb, self._outs, n, make_materials(materials), len(materials),
                                 make_lights(lights), len(lights),
                                 C.byref(make_params(k_max, n_probe_max, rounding)),
                                 C.byref(t) if t is not None else None, C.byref(h))
        _check(st, "glint_plan_create")
        self._h = h

    def run(self, use_graph=True, stream=None):
        _check(lib().glint_shade_batched(self._h, int(bool(use_graph)), _stream(stream)), "glint_shade_batched")

    def info(self):
        nt, nb = C.c_int64(), C.c_int32()
        _check(lib().glint_plan_info(self._h, C.byref(nt), C.byref(nb)), "glint_plan_info")
        return nt.value, nb.value

    def close(self):
        if getattr(self, "_h", None):
            lib().glint_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def glint_texel_hash(keys, stream=None):
    """keys: int32 CUDA tensor [n, 9] (seed, l, k, m, i, j, ai, aj, slot) -> uint32 as int32 [n]."""
    n = keys.shape[0]
    out = torch.empty(n, dtype=torch.int32, device=keys.device)
    _check(lib().glint_texel_hash(_dev_ptr(keys, torch.int32, "keys"), n, out.data_ptr(), _stream(stream)),
           "glint_texel_hash")
    return out


def glint_hash_step(h, w, stream=None):
    n = h.numel()
    out = torch.empty(n, dtype=torch.int32, device=h.device)
    _check(lib().glint_hash_step(_dev_ptr(h, torch.int32, "h"), _dev_ptr(w, torch.int32, "w"), n,
                                 out.data_ptr(), _stream(stream)), "glint_hash_step")
    return out


def glint_ndtri(bits, stream=None):
    n = bits.numel()
    out = torch.empty(n, dtype=torch.float32, device=bits.device)
    _check(lib().glint_ndtri(_dev_ptr(bits, torch.int32, "bits"), n, out.data_ptr(), _stream(stream)),
           "glint_ndtri")
    return out
