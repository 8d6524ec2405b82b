"""GPU parity of the random-number table variant (Sec. 6.3: the two uniforms
of a gated binomial read from a small precomputed texture) against the FP64
oracle's table mode, through the C ABI (glint_rng_table_fill,
glint_shade_rng_table).

Run on an MI355X:  python -u -m pytest tests -m gpu -x -v --timeout 120 --timeout-method thread
"""
import numpy as np
import pytest

import oracle
from paper_2306_05051_amd import scenes
from parity_util import compare, dbg_to_numpy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEED = 0x5EED


@pytest.fixture(scope="module")
def glint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_05051_amd import glint as g
    g.lib()
    return g


@pytest.mark.parametrize("log2,seed", [(8, 0), (12, SEED), (20, 0xFFFFFFFF)])
def test_table_entries_match_the_oracle(glint, log2, seed):
    print(f"  table 2^{log2} seed {seed:#x}", flush=True)
    t = glint.glint_rng_table_fill(log2, seed).cpu().numpy().view(np.uint32)
    n = 1 << log2
    idx = np.arange(n) if n <= 4096 else np.unique(np.r_[0, 1, n - 1, np.random.default_rng(log2).integers(0, n, 3000)])
    ref = np.array([oracle.rng_table_entry(seed, int(i)) for i in idx], dtype=np.uint32)
    assert np.array_equal(t[idx], ref)


def _shade_table(glint, dgb, mats, lights, table, log2, placement, **kw):
    rgb, dbg = glint.glint_shade_rng_table(dgb, mats, lights, table, log2, placement, debug=True, **kw)
    rgb2 = glint.glint_shade_rng_table(dgb, mats, lights, table, log2, placement, **kw)
    torch.cuda.synchronize()
    # the production kernel (gates that cannot open skipped) gives the debug kernel's bits
    assert torch.equal(rgb, rgb2)
    return rgb2, dbg


@pytest.mark.parametrize("log2", [8, 12, 16])
def test_table_parity_with_the_oracle(glint, log2):
    """Both placements against the oracle's table mode on a ragged 4K-like
    frame (8 materials, 4 lights, split footprints)."""
    gb, mats, lights = scenes.four_k(250, 141, seed=3)
    print(f"  table 2^{log2}: frame {gb['u'].shape}", flush=True)
    dgb = glint.to_device(gb)
    table = glint.glint_rng_table_fill(log2, SEED)
    rgb_c, dbg = _shade_table(glint, dgb, mats, lights, table, log2, glint.RNG_CACHED)
    if log2 <= glint.GLINT_RNG_LDS_MAX_LOG2:
        rgb_l, _ = _shade_table(glint, dgb, mats, lights, table, log2, glint.RNG_LDS)
        assert torch.equal(rgb_c, rgb_l)
    rrgb, rdbg = oracle.shade(gb, mats, lights, debug=True, rng_table=(log2, SEED))
    st = compare(rgb_c.cpu().numpy(), dbg_to_numpy(dbg), rrgb, rdbg, label=f"table 2^{log2}")
    print(f"  table 2^{log2}: {st}", flush=True)
    assert st["checked"] > 0.9 * st["shaded"] and st["nonzero"] > 100


def test_lds_placement_at_its_largest_table(glint):
    log2 = glint.GLINT_RNG_LDS_MAX_LOG2
    gb, mats, lights = scenes.sphere_forward(160, 90, seed=1)
    dgb = glint.to_device(gb)
    table = glint.glint_rng_table_fill(log2, 3)
    a = glint.glint_shade_rng_table(dgb, mats, lights, table, log2, glint.RNG_CACHED)
    b = glint.glint_shade_rng_table(dgb, mats, lights, table, log2, glint.RNG_LDS)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_full_width_table_is_the_hash_path(glint):
    """table[i] = H(0, i) over all 2^32 indices (16 GiB): reading it at
    texel key ^ angular key gives H(texel key, angular key), so the table
    variant must reproduce glint_shade bit for bit."""
    gb, mats, lights = scenes.four_k(128, 72, seed=5)
    dgb = glint.to_device(gb)
    ref = glint.glint_shade(dgb, mats, lights)
    table = glint.glint_rng_table_fill(32, 0)
    out = glint.glint_shade_rng_table(dgb, mats, lights, table, 32, glint.RNG_CACHED)
    torch.cuda.synchronize()
    assert float(ref.abs().sum()) > 0.0
    assert torch.equal(out, ref)
    del table
    torch.cuda.empty_cache()
