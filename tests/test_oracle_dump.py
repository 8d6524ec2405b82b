"""Pins of the oracle's sampled per-texel dump (CPU only).

The dump reports, per sampled pixel and probe, every texel-level value the
method draws: the simplex texel keys and barycentric weights of each grid
node (Secs. 4.3, 6.2), and per light and angular texel (Eq. 14) the word
behind the gate uniform (Eq. 18) and the count (Eq. 17).  These tests hold
it to the method from outside the oracle's own code:

* the words are hashes of (texel key, angular key): inverting the hash's
  finaliser (a bijection) recovers one angular key per light and angular
  texel, the same for every texel of every probe of the pixel; inverting it
  again gives the angular texel's indices, which must be the four texels
  around the half vector's projection on the supplied tangent frame,
  computed here in numpy from the G-buffer (lights below the horizon: all 0);
* the counts, weights and the bilinear angular weights computed here
  reconstruct the pixel's distributed count b of every light (Eq. 14 over
  the nodes' texels);
* the barycentric weights of each node are a partition of unity;
* sums over the dump equal the per-pixel fingerprints (key, gate-word and
  count sums, open gates), and every entry without a texel is 0.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2306_05051_amd import scenes

GOLDEN = 0x9E3779B9
ANG_SALT = 0x13198A2E
M32 = 0xFFFFFFFF


def _fmix_inv(h):
    """inverse of the MurmurHash3 finaliser (xor-shifts and odd multipliers)"""
    h = np.asarray(h, np.uint64) & M32
    i1, i2 = pow(0x85EBCA6B, -1, 1 << 32), pow(0xC2B2AE35, -1, 1 << 32)
    h ^= h >> 16
    h = (h * i2) & M32
    h ^= (h >> 13) ^ (h >> 26)
    h = (h * i1) & M32
    h ^= h >> 16
    return h


def _step_inv(out, h):
    """the word w with hash_step(h, w) == out"""
    return ((_fmix_inv(out) - GOLDEN) & M32) ^ (np.asarray(h, np.uint64) & M32)


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _scene(seed=3, W=48, H=24):
    g, mats, lights = scenes.four_k(W=W, H=H, seed=seed, n_light=3)
    rng = np.random.default_rng(77 + seed)
    t = rng.normal(size=(3, H, W))
    g["tx"], g["ty"], g["tz"] = [t[i].astype(np.float32) for i in range(3)]
    return g, mats, lights


def _pick(d, n, rng):
    """a mix of split, single-probe, and unshaded pixels"""
    shaded = (d["flags"] & 1) > 0
    split = np.argwhere(shaded & (d["n_probe"] > 1))
    single = np.argwhere(shaded & (d["n_probe"] == 1))
    other = np.argwhere(~shaded)
    pick = [split[rng.choice(len(split), min(n, len(split)), replace=False)],
            single[rng.choice(len(single), min(n, len(single)), replace=False)]]
    if len(other):
        pick.append(other[:2])
    return np.concatenate(pick)


def test_dump_words_counts_and_weights():
    g, mats, lights = _scene()
    _, d0 = oracle.shade(g, mats, lights, debug=True)
    yx = _pick(d0, 12, np.random.default_rng(5))
    P = 21
    _, d = oracle.shade(g, mats, lights, debug=True, dump_pixels=yx, dump_probes=P)
    dm = d["dump"]
    assert np.array_equal(dm["slot"][yx[:, 0], yx[:, 1]], np.arange(len(yx)))
    n_checked_light = 0
    for s, (y, x) in enumerate(yx):
        key, beta, theta, count = dm["key"][s], dm["beta"][s], dm["theta"][s], dm["count"][s]
        if not d["flags"][y, x] & 1:
            for a in (key, beta, theta, count):
                assert not np.any(a)
            continue
        npr, nn = int(d["n_probe"][y, x]), int((d["cell"][y, x] >> 15) & 7)
        assert 1 <= nn <= 4
        # no texel: 0
        for a in (key, beta, theta, count):
            assert not np.any(a[npr:])
            assert not np.any(a[:npr, ..., nn:, :] if a.ndim == 3 else a[:npr, :, nn:])
        # fingerprints
        assert int(key[:npr].astype(np.uint64).sum() & M32) == int(d["key_sum"][y, x])
        assert int(theta.astype(np.uint64).sum() & M32) == int(d["theta_sum"][y, x])
        assert int(np.count_nonzero(count)) == int(d["n_open"][y, x])
        assert int(count.sum()) == int(d["count_sum"][y, x])
        # partition of unity
        b = beta[:npr, :nn]
        assert np.all(b >= -1e-12)
        assert np.allclose(b.sum(-1), 1.0, atol=1e-12)
        # the angular texels, from outside: frame of the supplied tangent
        n = _unit([g["nx"][y, x], g["ny"][y, x], g["nz"][y, x]])
        wi = _unit([g["wx"][y, x], g["wy"][y, x], g["wz"][y, x]])
        t = np.array([g["tx"][y, x], g["ty"][y, x], g["tz"][y, x]], np.float64)
        t = _unit(t - np.dot(t, n) * n)
        bb = np.cross(n, t)
        # the oracle takes material and light values in FP32, as the ABI does
        mr = float(np.float32(mats[int(g["material_id"][y, x])]["micro_roughness"]))
        for li, L in enumerate(lights):
            wo = _unit(np.asarray(L["dir"], np.float32))
            th = theta[:npr, li, :nn]
            if np.dot(n, wo) <= 0.0:
                assert not np.any(th) and not np.any(count[:, li])
                continue
            h = _unit(wi + wo)
            ax, ay = np.dot(h, t) / mr - 0.5, np.dot(h, bb) / mr - 0.5
            if min(abs(ax - round(ax)), abs(ay - round(ay))) < 1e-9:
                continue                      # on a cell edge: the FP64 floors may differ
            ai, aj = math.floor(ax), math.floor(ay)
            fx, fy = ax - ai, ay - aj
            vw = np.array([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy])
            # one angular key per angular texel a, shared by every texel
            ak = _step_inv(th, key[:npr, :nn, :, None])
            for a in range(4):
                assert np.unique(ak[..., a]).size == 1, "angular key differs between texels"
                w = int(_step_inv(ak[0, 0, 0, a], ANG_SALT))
                A, B, slot = w & 0x7FFF, (w >> 15) & 0x7FFF, w >> 30
                assert slot == 0
                assert (A - 16384, B - 16384) == (ai + (a & 1), aj + (a >> 1)), (a, A, B, ai, aj)
            # Eq. 14 over the nodes' texels: the pixel's count sum b
            bl = float(np.sum(beta[:npr, :nn, :, None] * vw * count[:npr, li, :nn]))
            assert bl == pytest.approx(float(d["b_light"][li, y, x]), rel=1e-12, abs=1e-300)
            n_checked_light += 1
    assert n_checked_light >= 20


def test_dump_matches_fingerprints_zk_and_relaxed():
    g, mats, lights = _scene(seed=4)
    _, d0 = oracle.shade(g, mats, lights, debug=True)
    yx = _pick(d0, 8, np.random.default_rng(6))
    for kw in (dict(count_law=1), dict(rounding=1)):
        _, d = oracle.shade(g, mats, lights, debug=True, dump_pixels=yx, dump_probes=21, **kw)
        dm = d["dump"]
        for s, (y, x) in enumerate(yx):
            npr = int(d["n_probe"][y, x])
            assert int(dm["key"][s, :npr].astype(np.uint64).sum() & M32) == int(d["key_sum"][y, x])
            assert int(dm["theta"][s].astype(np.uint64).sum() & M32) == int(d["theta_sum"][y, x])
            if kw.get("count_law"):
                assert int(dm["count"][s].sum()) == int(d["count_sum"][y, x])
            else:
                # relaxed counts are real, at least 1 where a gate opened
                c = dm["count"][s]
                assert np.count_nonzero(c) == int(d["n_open"][y, x])
                assert np.all(c[c != 0] >= 1.0)


def test_dump_probe_cap():
    """dump_probes below n_probe keeps the pixel's first probes"""
    g, mats, lights = _scene(seed=5)
    _, d0 = oracle.shade(g, mats, lights, debug=True)
    yx = _pick(d0, 6, np.random.default_rng(7))
    _, full = oracle.shade(g, mats, lights, debug=True, dump_pixels=yx, dump_probes=21)
    _, cap = oracle.shade(g, mats, lights, debug=True, dump_pixels=yx, dump_probes=2)
    for k in ("key", "beta", "theta", "count"):
        assert np.array_equal(cap["dump"][k], full["dump"][k][:, :2])
