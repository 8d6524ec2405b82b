"""GPU parity of the sampled per-texel dump (glint_debug's dump arrays)
against the oracle's: texel keys, gate words and counts of every probe,
node, lattice vertex, light and angular texel of the sampled pixels.

Run on an MI355X:  python -u -m pytest tests -m gpu -x -v --timeout 120 --timeout-method thread
"""
import numpy as np
import pytest

import oracle
from paper_2306_05051_amd import scenes
from parity_util import compare_dump, dbg_to_numpy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def glint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_05051_amd import glint as g
    g.lib()
    return g


def _scene(W, H, seed, tangents=True):
    g, mats, lights = scenes.four_k(W=W, H=H, seed=seed)
    if tangents:
        rng = np.random.default_rng(90 + seed)
        t = rng.normal(size=(3, H, W))
        g["tx"], g["ty"], g["tz"] = [t[i].astype(np.float32) for i in range(3)]
    return g, mats, lights


def _sample(flags, n_probe, n, seed):
    """split, single-probe and unshaded pixels"""
    rng = np.random.default_rng(seed)
    shaded = (flags & 1) > 0
    groups = [np.argwhere(shaded & (n_probe > 1)), np.argwhere(shaded & (n_probe == 1)), np.argwhere(~shaded)]
    pick = [gr[rng.choice(len(gr), min(n, len(gr)), replace=False)] for gr in groups if len(gr)]
    return np.concatenate(pick)


@pytest.mark.parametrize("case", ["method", "relaxed", "zk_baseline", "onb_frame"])
def test_dump_parity(glint, case):
    kw = {"method": {}, "relaxed": dict(rounding=1), "zk_baseline": dict(count_law=1),
          "onb_frame": {}}[case]
    gb, mats, lights = _scene(96, 64, seed=11, tangents=case != "onb_frame")
    _, rd0 = oracle.shade(gb, mats, lights, debug=True, **kw)
    yx = _sample(rd0["flags"], rd0["n_probe"], 24, seed=3)
    P = 21
    print(f"  dump {case}: {len(yx)} pixels, {P} probes", flush=True)
    _, rd = oracle.shade(gb, mats, lights, debug=True, dump_pixels=yx, dump_probes=P, **kw)
    dgb = glint.to_device(gb)
    rgb, gd = glint.glint_shade(dgb, mats, lights, debug=True, dump_pixels=yx, dump_probes=P, **kw)
    rgb_plain = glint.glint_shade(dgb, mats, lights, **kw)
    torch.cuda.synchronize()
    # the dump does not change the image
    assert torch.equal(rgb, rgb_plain)
    gd = dbg_to_numpy(gd)
    n = compare_dump(gd["dump"], rd["dump"], rd, yx, relaxed=case == "relaxed", label=case)
    print(f"  {case}: {n} of {len(yx)} sampled pixels compared", flush=True)
    assert n >= 0.8 * len(yx)
    # the dump is not vacuous: gates opened in the compared pixels
    assert np.count_nonzero(gd["dump"]["count"]) > 0


def test_dump_probe_cap_and_rewrite(glint):
    """dump_probes below n_probe keeps the first probes; a second call into
    the same arrays rewrites every entry of its slots"""
    gb, mats, lights = _scene(64, 32, seed=12)
    _, rd0 = oracle.shade(gb, mats, lights, debug=True)
    yx = _sample(rd0["flags"], rd0["n_probe"], 8, seed=4)
    dgb = glint.to_device(gb)
    _, full = glint.glint_shade(dgb, mats, lights, debug=True, dump_pixels=yx, dump_probes=21)
    _, cap = glint.glint_shade(dgb, mats, lights, debug=True, dump_pixels=yx, dump_probes=3)
    torch.cuda.synchronize()
    for k in ("key", "beta", "theta", "count"):
        assert torch.equal(cap["dump"][k], full["dump"][k][:, :3])


def test_dump_full_4k_sampled_pixels(glint):
    """Dump of sampled pixels of the full 3840x2160 frame, compared with the
    oracle on their rows"""
    gb, mats, lights = scenes.four_k(3840, 2160, seed=3)
    rows = [7, 1080, 2159]
    rng = np.random.default_rng(8)
    yx = np.array([(r, int(x)) for r in rows for x in rng.choice(3840, 16, replace=False)])
    dgb = glint.to_device(gb)
    print("  full 4K frame dump", flush=True)
    _, gd = glint.glint_shade(dgb, mats, lights, debug=True, dump_pixels=yx, dump_probes=21)
    torch.cuda.synchronize()
    gd = dbg_to_numpy(gd)
    n = 0
    for i, r in enumerate(rows):
        sub = {k: v[r:r + 1] for k, v in gb.items()}
        sel = yx[yx[:, 0] == r]
        loc = np.stack([np.zeros(len(sel), np.int64), sel[:, 1]], 1)
        _, rd = oracle.shade(sub, mats, lights, debug=True, dump_pixels=loc, dump_probes=21)
        gsl = {k: gd["dump"][k][16 * i:16 * (i + 1)] for k in ("key", "beta", "theta", "count")}
        n += compare_dump(gsl, rd["dump"], rd, loc, label=f"4K row {r}")
    print(f"  4K: {n} of {len(yx)} sampled pixels compared", flush=True)
    assert n >= 0.8 * len(yx)
