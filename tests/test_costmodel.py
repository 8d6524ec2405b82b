"""The roofline's unit counts (costmodel.units_from_debug) against counts
made directly from the inputs, on the oracle's debug planes (the GPU's are
bit-identical to them on every compared pixel): a (pixel, light) pair is
credited once however many probes the pixel has, an item once per probe."""
import numpy as np

import oracle
from paper_2306_05051_amd import costmodel, scenes


def test_units_count_pixel_lights_once():
    gb, mats, lights = scenes.four_k(96, 64, seed=11, n_light=3)
    _, d = oracle.shade(gb, mats, lights, debug=True)
    u = costmodel.units_from_debug(d)
    shaded = (d["flags"] & 1) > 0
    n = np.stack([gb["nx"], gb["ny"], gb["nz"]]).astype(np.float64)
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    valid = np.zeros(shaded.shape, np.int64)
    for l in lights:
        wo = np.asarray(l["dir"], np.float64)
        wo /= np.linalg.norm(wo)
        valid += (np.einsum("chw,c->hw", n, wo) > 0.0) & shaded
    npr = d["n_probe"].astype(np.int64)
    assert u["pixel"] == int(shaded.sum())
    # items of the pixels where some gate can open (the others shade to 0)
    live_px = shaded & ((d["n_live"].astype(np.int64) & 0xFFFFFFFF) > 0)
    assert u["item"] == int(npr[live_px].sum()) and 0 < u["item"] <= int(npr[shaded].sum())
    assert u["pixel_light"] == int(valid.sum())
    assert u["item_light"] == int((valid * npr).sum())
    # split footprints make the difference: more item-lights than pixel-lights
    assert u["item_light"] > 1.5 * u["pixel_light"]
    assert 0 < u["pixel_light_lit"] <= u["pixel_light"]
    assert u["live_gate"] + u["live_gate_small"] <= u["gate"]
    assert set(costmodel.COST) <= set(u)
    s = costmodel.slots(u)
    assert s == sum(costmodel.COST[k] * u[k] for k in costmodel.COST) and s > 0
