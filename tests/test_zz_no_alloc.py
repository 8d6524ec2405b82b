"""glint_shade_noalloc, the entry point that allocates nothing (its tile-order
workspace is the library's static device array), against glint_shade with a
caller-owned workspace: the same image bit for bit (the same kernels and tile
order), over two calls in a row on the same GPU, the second on a smaller view
so that it reuses the array left by the first.  Also: the size limit is
rejected before any launch.

Run on an MI355X:  python -u -m pytest tests/test_zz_no_alloc.py -x -v --timeout 120 --timeout-method thread
"""
import ctypes as C

import numpy as np
import pytest

from paper_2306_05051_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def glint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_05051_amd import glint as g
    g.lib()
    return g


def _pair(glint, W, H, seed, **kw):
    print(f"  no-alloc vs workspace: {W}x{H} seed={seed} {kw}", flush=True)
    gb, mats, lights = scenes.four_k(W, H, seed=seed, n_light=3)
    dgb = glint.to_device(gb)
    out = torch.full((3, H, W), float("nan"), dtype=torch.float32, device="cuda")
    a = glint.glint_shade_noalloc(dgb, mats, lights, out=out, **kw)
    b = glint.glint_shade(dgb, mats, lights, **kw)                   # caller-owned workspace
    c = glint.glint_shade(dgb, mats, lights, workspace=False, **kw)  # row-major tiles, no workspace
    torch.cuda.synchronize()
    assert a.data_ptr() == out.data_ptr()
    assert torch.isfinite(a).all()
    assert torch.equal(a, b), f"{W}x{H}: differs from glint_shade with a workspace"
    assert torch.equal(a, c), f"{W}x{H}: differs from glint_shade without a workspace"
    assert (a[0] > 0).sum().item() > 0.01 * W * H, "vacuous comparison: almost nothing lit"
    return a


def test_noalloc_two_calls_second_smaller(glint):
    _pair(glint, 1920, 1080, seed=21)
    _pair(glint, 333, 177, seed=22)          # smaller and ragged: reuses the first call's array
    _pair(glint, 333, 177, seed=22, rounding=1)


def test_noalloc_zk_law_and_empty(glint):
    _pair(glint, 257, 131, seed=23, count_law=glint.LAW_ZK)
    g = glint._GBuf()
    g.width, g.height, g.stride = 0, 5, 0
    mats = glint.make_materials([dict(alpha=0.3, log10_density=5.0)])
    lts = glint.make_lights([dict(dir=(0, 0, 1))])
    st = glint.lib().glint_shade_noalloc(C.byref(g), mats, 1, lts, 1, C.byref(glint.make_params()), None, None)
    assert st == glint.GLINT_OK


def test_noalloc_rejects_views_beyond_the_static_workspace(glint):
    L = glint.lib()
    mats = glint.make_materials([dict(alpha=0.3, log10_density=5.0)])
    lts = glint.make_lights([dict(dir=(0, 0, 1))])
    prm = glint.make_params()
    g = glint._GBuf()
    g.width, g.height, g.stride = 8192, 4096, 8192
    assert L.glint_shade_workspace_bytes(8192, 4096) > glint.GLINT_NOALLOC_WORKSPACE_BYTES
    assert L.glint_shade_noalloc(C.byref(g), mats, 1, lts, 1, C.byref(prm), None, None) == glint.GLINT_ELIMIT
    assert L.glint_shade_workspace_bytes(5120, 4096) <= glint.GLINT_NOALLOC_WORKSPACE_BYTES
