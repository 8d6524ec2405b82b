"""GPU adjoint (glint_shade_backward, through the C ABI and the autograd
Function) against the FP64 oracle's two gradients -- central differences with
the branches frozen, and forward-mode dual numbers -- and against GPU central
differences of the relaxed forward."""
import math

import numpy as np
import pytest

import oracle
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


def _close(a, b, rtol, label):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    scale = np.abs(b).max()
    err = np.abs(a - b)
    assert np.all(err <= rtol * np.abs(b) + 0.02 * rtol * scale + 1e-30), (label, a, b, err / np.maximum(np.abs(b), 1e-30))


def _loss_grad_out(glint, gb, mats, lights, tmats, tlights):
    """grad_out = L - L_target of the loss 1/2 sum (L - L_t)^2 (relaxed counts)."""
    dgb = glint.to_device(gb)
    L = glint.glint_shade(dgb, mats, lights, rounding=1)
    Lt = glint.glint_shade(dgb, tmats, tlights, rounding=1)
    torch.cuda.synchronize()
    return dgb, (L - Lt).contiguous()


@pytest.mark.parametrize("size,seed", [((96, 96), 2), ((160, 120), 3)])
def test_adjoint_matches_oracle_gradient(glint, size, seed):
    gb, mats, lights, tmats, tlights = scenes.backward_scene(size[0], size[1], seed=seed)
    dgb, go = _loss_grad_out(glint, gb, mats, lights, tmats, tlights)
    ga, gn, gd = glint.glint_shade_backward(dgb, mats, lights, go)
    torch.cuda.synchronize()
    ra, rn, rd, _ = oracle.grad(gb, mats, lights, go.cpu().numpy().astype(np.float64), step=1e-6, frozen=True)
    print("  gpu", ga.cpu().numpy(), gn.cpu().numpy(), gd.cpu().numpy().ravel())
    print("  fp64", ra, rn, rd.ravel())
    _close(ga.cpu().numpy(), ra, 1e-3, "alpha")
    _close(gn.cpu().numpy(), rn, 1e-3, "lnN")
    _close(gd.cpu().numpy(), rd, 1e-3, "dir")
    # the dual-number gradient: no step size, no shared code with the above
    ja, jn, jd, _ = oracle.grad_dual(gb, mats, lights, go.cpu().numpy().astype(np.float64))
    _close(ga.cpu().numpy(), ja, 1e-3, "alpha (dual)")
    _close(gn.cpu().numpy(), jn, 1e-3, "lnN (dual)")
    _close(gd.cpu().numpy(), jd, 1e-3, "dir (dual)")


def test_adjoint_multi_material_multi_light(glint):
    gb, mats, lights = scenes.four_k(96, 64, seed=9, n_light=3, n_mat=4)
    rng = np.random.default_rng(0)
    go = rng.normal(size=(3,) + gb["u"].shape).astype(np.float32)
    dgb = glint.to_device(gb)
    ga, gn, gd = glint.glint_shade_backward(dgb, mats, lights, torch.from_numpy(go).cuda())
    torch.cuda.synchronize()
    ra, rn, rd, _ = oracle.grad(gb, mats, lights, go.astype(np.float64), step=1e-6, frozen=True)
    _close(ga.cpu().numpy(), ra, 2e-3, "alpha")
    _close(gn.cpu().numpy(), rn, 2e-3, "lnN")
    _close(gd.cpu().numpy(), rd, 2e-3, "dir")
    ja, jn, jd, _ = oracle.grad_dual(gb, mats, lights, go.astype(np.float64))
    _close(ga.cpu().numpy(), ja, 2e-3, "alpha (dual)")
    _close(gn.cpu().numpy(), jn, 2e-3, "lnN (dual)")
    _close(gd.cpu().numpy(), jd, 2e-3, "dir (dual)")


def test_autograd_function_and_gpu_central_differences(glint):
    from paper_2306_05051_amd.autograd import GlintShade
    gb, mats, lights, tmats, tlights = scenes.backward_scene(128, 128, seed=4)
    dgb = glint.to_device(gb)
    Lt = glint.glint_shade(dgb, tmats, tlights, rounding=1)
    a = torch.tensor([mats[0]["alpha"]], dtype=torch.float64, requires_grad=True)
    n = torch.tensor([mats[0]["log10_density"] * math.log(10.0)], dtype=torch.float64, requires_grad=True)
    d = torch.tensor([lights[0]["dir"]], dtype=torch.float64, requires_grad=True)
    L = GlintShade.apply(a, n, d, dgb, mats, lights)
    loss = 0.5 * ((L - Lt) ** 2).double().sum()
    loss.backward()
    # central differences of the same loss with the GPU forward, on pixels whose
    # branches do not flip: compare against the adjoint restricted to them is not
    # possible per pixel, so use steps small enough that flips are rare and
    # check agreement to a looser bound
    def f(av, nv, dv):
        m = [dict(mats[0], alpha=av, log10_density=nv / math.log(10.0))]
        lt = [dict(lights[0], dir=tuple(dv))]
        Lx = glint.glint_shade(dgb, m, lt, rounding=1)
        return 0.5 * float(((Lx - Lt).double() ** 2).sum())
    a0, n0, d0 = float(a), float(n), list(d.detach().numpy()[0])
    h = 1e-4
    fd_a = (f(a0 + h, n0, d0) - f(a0 - h, n0, d0)) / (2 * h)
    fd_n = (f(a0, n0 + h, d0) - f(a0, n0 - h, d0)) / (2 * h)
    print("  adjoint", a.grad.item(), n.grad.item(), d.grad.numpy(), " fd", fd_a, fd_n)
    assert a.grad.item() == pytest.approx(fd_a, rel=0.05)
    assert n.grad.item() == pytest.approx(fd_n, rel=0.05)
    # the oracle's frozen gradient on the same loss
    ra, rn, rd, _ = oracle.grad(gb, mats, lights, (L - Lt).detach().cpu().numpy().astype(np.float64),
                                step=1e-6, frozen=True)
    _close([a.grad.item()], ra, 1e-3, "alpha")
    _close([n.grad.item()], rn, 1e-3, "lnN")
    _close(d.grad.numpy(), rd, 1e-3, "dir")


def test_backward_deterministic_and_errors(glint):
    gb, mats, lights, _, _ = scenes.backward_scene(64, 48, seed=6)
    dgb = glint.to_device(gb)
    go = torch.randn((3, 48, 64), device="cuda")
    r1 = glint.glint_shade_backward(dgb, mats, lights, go)
    r2 = glint.glint_shade_backward(dgb, mats, lights, go)
    torch.cuda.synchronize()
    for x, y in zip(r1, r2):
        assert torch.equal(x, y)
    g2 = dict(dgb)
    g2["alpha_px"] = torch.full_like(dgb["u"], 0.3)
    with pytest.raises(glint.GlintError) as e:
        glint.glint_shade_backward(g2, mats, lights, go)
    assert e.value.status == glint.GLINT_EUNSUPPORTED


def _lit_cases():
    return [("backward 128x96", lambda: scenes.backward_scene(128, 96, seed=7)[:3]),
            ("4k-like 3 lights", lambda: scenes.four_k(96, 64, seed=9, n_light=3, n_mat=4)),
            ("4k-like 16 lights", lambda: scenes.four_k(64, 40, seed=11, n_light=16, n_mat=5)),
            ("paper plane25", lambda: scenes.paper_setting(160, 90, view="plane25", log10_density=6.0, seed=3)),
            ("wide rows", lambda: scenes.four_k(2100, 12, seed=13, n_light=2, n_mat=3))]


@pytest.mark.parametrize("case", range(5))
def test_lit_mask_matches_oracle(glint, case):
    """glint_shade_lit: radiance identical to glint_shade, and per pixel the set
    of lights with an open gate equals the oracle's on every compared pixel."""
    from parity_util import MARGIN
    label, make = _lit_cases()[case]
    gb, mats, lights = make()
    print(f"  {label}: {gb['u'].shape}, {len(lights)} lights", flush=True)
    dgb = glint.to_device(gb)
    out, lit, probes = glint.glint_shade_lit(dgb, mats, lights, rounding=1)
    ref, gdbg = glint.glint_shade(dgb, mats, lights, rounding=1, debug=True)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    g = lit.cpu().numpy().view(np.uint16).astype(np.uint32)
    # the probe mask: non-empty exactly where a light is lit, within the pixel's probes
    pm = probes.cpu().numpy().view(np.uint32).astype(np.int64)
    npr = gdbg["n_probe"].cpu().numpy().astype(np.int64)
    assert np.array_equal(pm != 0, g != 0)
    assert np.all(pm < (np.int64(1) << np.minimum(npr, 32)))
    _, d = oracle.shade(gb, mats, lights, rounding=1, debug=True)
    shaded = (d["flags"] & 1) > 0
    ok = shaded & (d["margin_pos"] >= MARGIN)
    assert np.all(g[~shaded] == 0)
    assert np.array_equal(g[ok], d["lit"][ok])
    assert np.count_nonzero(g) > 20
    print(f"  {label}: {np.count_nonzero(g)} of {shaded.sum()} shaded pixels lit, "
          f"{int(np.unpackbits(g.view(np.uint8)).sum())} lit pixel-lights", flush=True)


@pytest.mark.parametrize("case", range(5))
def test_backward_with_lit_mask_matches_full_adjoint(glint, case):
    """The adjoint that shades only the lit pixels (gathered into full waves) and
    their lit lights adds the same terms as the full adjoint, grouped into other
    waves and partial rows: equal within FP32 rounding, and deterministic."""
    label, make = _lit_cases()[case]
    gb, mats, lights = make()
    dgb = glint.to_device(gb)
    _, lit, probes = glint.glint_shade_lit(dgb, mats, lights, rounding=1)
    go = torch.randn((3,) + gb["u"].shape, device="cuda", generator=torch.Generator("cuda").manual_seed(case))
    full = glint.glint_shade_backward(dgb, mats, lights, go)
    fast = glint.glint_shade_backward(dgb, mats, lights, go, lit=lit)
    fastest = glint.glint_shade_backward(dgb, mats, lights, go, lit=lit, probes=probes)
    torch.cuda.synchronize()
    print(f"  {label}: grad alpha {full[0].cpu().numpy()}", flush=True)
    for res in (fast, fastest):
        for a, b in zip(full, res):
            a, b = a.double(), b.double()
            assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max()) + 1e-30
    assert float(full[0].abs().sum()) > 0.0
    # the masked adjoint is deterministic too
    again = glint.glint_shade_backward(dgb, mats, lights, go, lit=lit, probes=probes)
    torch.cuda.synchronize()
    for x, y in zip(fastest, again):
        assert torch.equal(x, y)


def test_backward_units_expand_probes_beyond_31(glint):
    """Footprints split into more than 31 probes: bit 31 of the probe mask
    stands for probes 31 on, and the masked adjoint (work units of
    (pixel, lit probe, lit light) items) expands it from the pixel's own probe
    count: the same gradient as the adjoint without masks."""
    gb, mats, lights = scenes.four_k(128, 48, seed=14, n_light=3, n_mat=3, n_probe_max=64)
    dgb = glint.to_device(gb)
    _, lit, probes = glint.glint_shade_lit(dgb, mats, lights, rounding=1, n_probe_max=64)
    go = torch.randn((3,) + gb["u"].shape, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    full = glint.glint_shade_backward(dgb, mats, lights, go, n_probe_max=64)
    fast = glint.glint_shade_backward(dgb, mats, lights, go, n_probe_max=64, lit=lit, probes=probes)
    torch.cuda.synchronize()
    beyond = int(((probes.cpu().numpy().view(np.uint32) >> 31) & 1).sum())
    print(f"  pixels with a lit probe from 31 on: {beyond}", flush=True)
    assert beyond > 0
    for a, b in zip(full, fast):
        a, b = a.double(), b.double()
        assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max()) + 1e-30


def test_backward_with_empty_lit_mask_is_zero(glint):
    """A mask with no lit pixel leaves nothing to differentiate: zero gradients."""
    gb, mats, lights = scenes.four_k(300, 7, seed=12, n_light=2, n_mat=2)
    dgb = glint.to_device(gb)
    lit = torch.zeros(gb["u"].shape, dtype=torch.int16, device="cuda")
    go = torch.ones((3,) + gb["u"].shape, device="cuda")
    ga, gn, gd = glint.glint_shade_backward(dgb, mats, lights, go, lit=lit)
    torch.cuda.synchronize()
    assert float(ga.abs().sum()) == 0.0 and float(gn.abs().sum()) == 0.0 and float(gd.abs().sum()) == 0.0
    full = glint.glint_shade_backward(dgb, mats, lights, go)
    _, lit2, probes2 = glint.glint_shade_lit(dgb, mats, lights, rounding=1)
    fast = glint.glint_shade_backward(dgb, mats, lights, go, lit=lit2, probes=probes2)
    torch.cuda.synchronize()
    for a, b in zip(full, fast):
        a, b = a.double(), b.double()
        assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max()) + 1e-30


def test_backward_empty_image_overwrites_gradients(glint):
    """An empty image has zero gradients, written over whatever the outputs
    held (a zeroing kernel, so the call stays capturable)."""
    import ctypes as C
    gb, mats, lights = scenes.four_k(32, 8, seed=2, n_light=3, n_mat=2)
    dgb = glint.to_device(gb)
    g = glint.make_gbuffer(dgb)
    g.width = 0
    ga = torch.full((2,), float("nan"), device="cuda")
    gn = torch.full((2,), float("nan"), device="cuda")
    gd = torch.full((3, 3), float("nan"), device="cuda")
    go = torch.zeros((3, 8, 32), device="cuda")
    st = glint.lib().glint_shade_backward(C.byref(g), glint.make_materials(mats), 2, glint.make_lights(lights), 3,
                                          C.byref(glint.make_params(rounding=1)), go.data_ptr(), None, None,
                                          ga.data_ptr(), gn.data_ptr(), gd.data_ptr(), None, 0, None)
    torch.cuda.synchronize()
    assert st == glint.GLINT_OK
    for t in (ga, gn, gd):
        assert torch.equal(t, torch.zeros_like(t))
