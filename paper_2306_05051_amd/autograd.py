"""torch.autograd.Function over glint_shade / glint_shade_backward.

    L = GlintShade.apply(alpha, ln_density, light_dir, gbuf, materials, lights)

alpha, ln_density: tensors [n_mat] (roughness, natural log of flakes per unit
UV area); light_dir: tensor [n_light, 3] (raw directions).  The forward
renders with relaxed counts (max(1, 1 + mu + sigma z), no floor) and records
which lights and probes opened a gate in each pixel; the backward is the
library's adjoint kernel, with every discrete branch held at its value at the
current parameters, skipping the pixels, probes and lights without an open
gate.  The parameter values are read on the host (the
library takes materials and lights by value), so the call synchronises once.
"""
from __future__ import annotations

import math

import torch

from . import glint


def _materials(base, alpha, ln_density):
    a = alpha.detach().double().cpu().tolist()
    n = ln_density.detach().double().cpu().tolist()
    return [dict(m, alpha=a[i], log10_density=n[i] / math.log(10.0)) for i, m in enumerate(base)]


def _lights(base, light_dir):
    d = light_dir.detach().double().cpu().tolist()
    return [dict(l, dir=tuple(d[i])) for i, l in enumerate(base)]


class GlintShade(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, ln_density, light_dir, gbuf, materials, lights, k_max=4, n_probe_max=21):
        mats = _materials(materials, alpha, ln_density)
        lts = _lights(lights, light_dir)
        out, lit, probes = glint.glint_shade_lit(gbuf, mats, lts, k_max=k_max, n_probe_max=n_probe_max, rounding=1)
        ctx.gbuf, ctx.mats, ctx.lts, ctx.lit, ctx.probes = gbuf, mats, lts, lit, probes
        ctx.k_max, ctx.n_probe_max = k_max, n_probe_max
        ctx.like = (alpha, ln_density, light_dir)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        ga, gn, gd = glint.glint_shade_backward(ctx.gbuf, ctx.mats, ctx.lts, grad_out.float().contiguous(),
                                                k_max=ctx.k_max, n_probe_max=ctx.n_probe_max, lit=ctx.lit,
                                                probes=ctx.probes)
        a, n, d = ctx.like
        return (ga.to(device=a.device, dtype=a.dtype), gn.to(device=n.device, dtype=n.dtype),
                gd.to(device=d.device, dtype=d.dtype), None, None, None, None, None)


def glint_shade_relaxed(alpha, ln_density, light_dir, gbuf, materials, lights, k_max=4, n_probe_max=21):
    return GlintShade.apply(alpha, ln_density, light_dir, gbuf, materials, lights, k_max, n_probe_max)
