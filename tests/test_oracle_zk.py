"""Pins of the oracle's Zirr-Kaplanyan counting baseline (CPU only).

The baseline is the prior art the paper replaces: the classical binomial
approximation (Sec. 6.3, Eq. 15: a Gaussian with the binomial's two moments,
floored, when n p > 5, else a loop of Bernoulli trials, at most 16 of them,
Sec. 7) and a linear mix of the binomial outputs of the grids that enclose the
footprint (Sec. 2, Eq. 7).  Pinned here against what mathematics fixes:

* the Bernoulli branch draws exactly Binomial(t, p) with t = floor(n + 1/2);
* the Gaussian branch's pmf equals the closed form through Phi
  (P(c = 0) = Phi((1 - mu)/sigma), P(c = j) = Phi((j + 1 - mu)/sigma) -
  Phi((j - mu)/sigma)), integrated on a stratified grid of uniforms;
* the branch switch sits at n p = 5 and n = 16;
* a pixel's mixed count has mean sum_g w_g E[c_g] and variance
  sum_g w_g^2 Var[c_g]: with the isotropic family (k_max = 0) the nodes are
  the two LOD levels of Eq. 7, and at mid-blend the variance falls to about
  half of the flake model's N P p (1 - p), the incorrect statistics Sec. 2
  predicts for this interpolation, while the distributed law keeps it;
* ghost flakes: at a lattice point the method counts whole flakes at every
  footprint area, the baseline shows half-intensity flakes at mid-blend.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle

R = 0.034
MICRO = 0.02


def _words(n, salt=0xA5A5):
    return [oracle.hash_step(salt, i) for i in range(n)]


@pytest.mark.parametrize("n,p", [(10.0, 0.3), (16.0, 0.25), (3.4, 0.9), (6.2, 0.05), (12.49, 0.4)])
def test_bernoulli_branch_is_binomial(n, p):
    M = 20000
    t = int(math.floor(n + 0.5))
    c = np.empty(M)
    for i, h in enumerate(_words(M)):
        c[i], g, tr = oracle.zk_count(n, p, h)
        assert g == 0 and tr == t
    assert np.all(c == np.floor(c)) and c.min() >= 0 and c.max() <= t
    obs = np.bincount(c.astype(int), minlength=t + 1)
    exp = stats.binom.pmf(np.arange(t + 1), t, p) * M
    keep = exp > 5
    chi2 = float(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]))
    assert stats.chi2.sf(chi2, max(1, keep.sum() - 1)) > 1e-4, (obs, exp)
    assert abs(c.mean() - t * p) < 5 * math.sqrt(t * p * (1 - p) / M) + 1e-12


@pytest.mark.parametrize("n,p", [(200.0, 0.1), (1e4, 1e-4), (17.0, 0.2), (5e5, 0.02)])
def test_gaussian_branch_matches_closed_form(n, p):
    mu, sd = n * p, math.sqrt(n * p * (1 - p))
    step = 64
    ks = np.arange(0, 1 << 23, step, dtype=np.int64)
    c = np.empty(ks.size)
    for i, k in enumerate(ks):
        c[i], g, tr = oracle.zk_count(n, p, int(k) << 9)
        assert g == 1 and tr == 0
    # stratified uniforms: the histogram integrates the pmf with resolution step / 2^23
    vals, cnt = np.unique(c, return_counts=True)
    hist = cnt / ks.size
    lo = np.where(vals == 0, -np.inf, (vals - mu) / sd)
    pmf = special.ndtr((vals + 1 - mu) / sd) - special.ndtr(lo)
    assert np.all(np.abs(hist - pmf) < 4.0 * step / (1 << 23) + 2e-3 * pmf), (vals, hist, pmf)
    # every count whose probability exceeds two grid cells is drawn
    j = np.arange(0, int(mu + 8 * sd) + 2)
    pj = special.ndtr((j + 1 - mu) / sd) - special.ndtr(np.where(j == 0, -np.inf, (j - mu) / sd))
    assert set(j[pj > 2.0 * step / (1 << 23)].tolist()) <= set(vals.astype(int).tolist())


def test_branch_switch():
    h = oracle.hash_step(7, 9)
    cases = [(16.0, 0.3125 - 1e-9, 0), (16.0, 0.3125 + 1e-9, 1), (16.4, 0.01, 1), (15.9, 0.01, 0),
             (100.0, 0.01, 1), (10.0, 0.5 + 1e-9, 1), (10.0, 0.5 - 1e-9, 0), (0.3, 0.9, 0)]
    for n, p, gauss in cases:
        c, g, t = oracle.zk_count(n, p, h)
        assert g == gauss, (n, p)
        assert t == (0 if gauss else int(math.floor(n + 0.5)))
    # no trials: nothing to count
    assert oracle.zk_count(0.3, 0.9, h)[0] == 0.0
    # on the Gaussian branch the count is the floored quantile, clamped at 0
    for k in (0, 1, 5000, (1 << 23) - 1, 4567890):
        n, p = 300.0, 0.05
        x = n * p + math.sqrt(n * p * (1 - p)) * special.ndtri((2 * k + 1) * 2.0**-24)
        assert oracle.zk_count(n, p, k << 9)[0] == max(0.0, math.floor(x))


def _pixel_sample(S, P, logN, count_law, k_max):
    from tests.test_oracle_statistics import _light_for_h, _single_pixel_gbuf
    s = math.sqrt(P)
    J = [[s, 0.0], [0.0, s]]
    g = _single_pixel_gbuf(S, (0.0, 0.0), J)
    wo, h = _light_for_h(0.999)
    alpha = 0.4
    mats = [dict(ndf=0, alpha=alpha, R=R, log10_density=logN, micro_roughness=MICRO, F0=1.0, seed=i)
            for i in range(S)]
    lights = [dict(dir=tuple(wo), radiance=(1, 1, 1))]
    _, dbg = oracle.shade(g, mats, lights, debug=True, k_max=k_max, count_law=count_law)
    J32 = [[float(np.float32(v)) for v in row] for row in J]
    fp = oracle.footprint(J32[0][0], J32[1][0], J32[0][1], J32[1][1])
    nodes, _, _ = oracle.grid_nodes(fp[0], fp[1], fp[2], k_max)
    w32 = np.array(wo, np.float32).astype(np.float64)
    h32 = np.array([0.0, 0.0, 1.0]) + w32 / np.linalg.norm(w32)
    h32 /= np.linalg.norm(h32)
    p = R * oracle.ndf(0, alpha, h32[2]) / oracle.ndf(0, alpha, 1.0)
    N = 10.0 ** np.float64(np.float32(logN))
    return dbg, nodes, p, N, fp[0]


def _floored_gauss_moments(n, p):
    mu, sd = n * p, math.sqrt(n * p * (1 - p))
    j = np.arange(0, int(mu + 12 * sd) + 2)
    lo = np.where(j == 0, -np.inf, (j - mu) / sd)
    pmf = special.ndtr((j + 1 - mu) / sd) - special.ndtr(lo)
    m = float(np.sum(j * pmf))
    return m, float(np.sum(j * j * pmf)) - m * m


def test_pixel_mix_of_outputs_and_its_variance_deficit():
    """Eq. 7 with the isotropic family: two LOD levels, weights (1 - t, t)."""
    S = 6000
    P = 1.5 * 2.0**-20                       # mid-blend: t = (P - 2^l) / 2^l = 1/2
    dbg, nodes, p, N, Pf = _pixel_sample(S, P, 9.0, 1, 0)
    assert [nd[0] for nd in nodes] == [-20, -19]
    assert [nd[3] for nd in nodes] == pytest.approx([0.5, 0.5], abs=1e-6)
    b = dbg["b_light"][0, 0]
    assert np.all(dbg["n_live"] == 0) and np.all(dbg["n_open"] == 24)      # Gaussian branch everywhere
    mom = [_floored_gauss_moments(N * 2.0**l, p) for (l, k, m, w) in nodes]
    mean_pred = sum(w * mm for (l, k, m, w), (mm, _) in zip(nodes, mom))
    var_pred = sum(w * w * vv for (l, k, m, w), (_, vv) in zip(nodes, mom))
    se = math.sqrt(var_pred / S)
    assert abs(b.mean() - mean_pred) < 5 * se, (b.mean(), mean_pred)
    assert b.var() == pytest.approx(var_pred, rel=8 * math.sqrt(2.0 / S) + 0.02)
    # the flake model: mean N P p (the mix keeps it, up to the floor's -1/2), variance N P p (1 - p)
    flake_var = N * Pf * p * (1 - p)
    assert abs(b.mean() - N * Pf * p) < 0.6 + 5 * se
    ratio = var_pred / flake_var
    assert ratio == pytest.approx(sum(w * w * 2.0**l for (l, k, m, w) in nodes)
                                  / sum(w * 2.0**l for (l, k, m, w) in nodes), rel=0.01)
    assert b.var() / flake_var < 0.6                        # about half: the predicted deficit
    # the distributed law on the same pixels keeps the binomial's spread
    dbg0, _, _, _, _ = _pixel_sample(S, P, 9.0, 0, 0)
    b0 = dbg0["b_light"][0, 0]
    assert b0.var() / flake_var == pytest.approx(1.0, rel=0.1)


def test_mixed_branches_count_trials():
    """A pixel whose lower level takes the Bernoulli loop and upper level the
    Gaussian: the debug planes count trials and Gaussian draws per texel."""
    S = 64
    P = 1.5 * 2.0**-20
    dbg, nodes, p, N, _ = _pixel_sample(S, P, 7.0, 1, 0)
    n_lo, n_hi = N * 2.0**-20, N * 2.0**-19
    assert n_lo <= 16 and n_lo * p <= 5 and n_hi > 16
    t = int(math.floor(n_lo + 0.5))
    assert np.all(dbg["n_live"] == 12 * t)
    assert np.all(dbg["n_open"] == 12)
    assert np.all(dbg["n_gate"] == 24)


def test_baseline_needs_integer_counts():
    from tests.test_oracle_statistics import _single_pixel_gbuf
    g = _single_pixel_gbuf(2, (0.0, 0.0), [[1e-3, 0.0], [0.0, 1e-3]])
    mats = [dict(ndf=0, alpha=0.3, R=R, log10_density=6.0, micro_roughness=MICRO, F0=1.0, seed=i)
            for i in range(2)]
    lights = [dict(dir=(0.1, 0.0, 1.0), radiance=(1, 1, 1))]
    with pytest.raises(ValueError):
        oracle.shade(g, mats, lights, rounding=1, count_law=1)
    with pytest.raises(ValueError):
        oracle.shade(g, mats, lights, count_law=2)


def test_ghost_flakes_at_mid_blend():
    """Sec. 2's ghosting: mixing the outputs of two LOD levels shows flakes at
    fractional intensity.  At a lattice-aligned point (one texel per node) the
    method's count is a whole number of flakes at every footprint area; the
    baseline's is (1 - t) c_lo + t c_hi, half-integers at mid-blend whenever
    the two levels disagree in parity."""
    S = 2000
    P = 1.5 * 2.0**-20
    dbg0, _, _, _, _ = _pixel_sample(S, P, 9.0, 0, 0)
    b0 = dbg0["b_light"][0, 0]
    # one angular texel carries (almost) all the weight: distance to the nearest integer is tiny
    assert np.max(np.abs(b0 - np.round(b0))) < 1e-3 * np.max(b0)
    dbg1, _, _, _, _ = _pixel_sample(S, P, 9.0, 1, 0)
    b1 = dbg1["b_light"][0, 0]
    frac = np.abs(b1 - np.round(b1))
    ghost = np.mean(frac > 0.25)
    assert 0.35 < ghost < 0.65, ghost       # about half the pixels show a half-intensity flake
