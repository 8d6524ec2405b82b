"""Explicit flake simulation and closed-form statistics -- TEST INFRASTRUCTURE ONLY.

These are the references the FP64 oracle is pinned to; none of them shares
code with the oracle's C implementation.

* ``stratified_counts``: the flake model the distributed binomial law is
  built to reproduce (Sec. 4.1, stratified distribution): one flake per fine
  cell of area 1/N, jittered uniformly inside its cell, each one reflecting
  with an explicit Bernoulli(p) trial.  A flake is a glint when it lies in the
  footprint and its trial succeeds (a spatialised Bernoulli trial).  Counting
  glints inside an arbitrary footprint (partial cells included) gives mean
  N P p exactly and a variance between N P p (1-p) and N P p.

* ``gated_pmf`` / ``gated_moments``: the distribution of the gated Gaussian
  binomial approximation (Sec. 6.3, Eqs. 16-18) in closed form through the
  normal CDF, under the reading used by the oracle: the gate succeeds when
  theta0 < P>=1, and an open gate gives max(1, floor(1 + mu + sigma Z)).
"""
from __future__ import annotations

import numpy as np
from scipy.stats import norm


def stratified_counts(N, footprint_inside, p, n_real, rng, box):
    """Count glints inside a footprint for n_real independent flake layouts.

    N: flakes per unit area (fine cells are squares of side 1/sqrt(N)).
    footprint_inside(x, y) -> bool mask, vectorised.
    box: (x0, x1, y0, y1) bounding box of the footprint.
    Returns an int array of n_real counts."""
    h = 1.0 / np.sqrt(N)
    i0, i1 = int(np.floor(box[0] / h)) - 1, int(np.ceil(box[1] / h)) + 1
    j0, j1 = int(np.floor(box[2] / h)) - 1, int(np.ceil(box[3] / h)) + 1
    ii, jj = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    out = np.zeros(n_real, np.int64)
    for r in range(n_real):
        x = (ii + rng.uniform(0, 1, ii.size)) * h
        y = (jj + rng.uniform(0, 1, jj.size)) * h
        inside = footprint_inside(x, y)
        reflect = rng.uniform(0, 1, ii.size) < p
        out[r] = int(np.count_nonzero(inside & reflect))
    return out


def coverage_fractions(N, footprint_inside, box, sub=64):
    """Fraction f_t of each fine cell covered by the footprint (sub x sub
    supersampling); the glint count is a sum of Bernoulli(f_t p)."""
    h = 1.0 / np.sqrt(N)
    i0, i1 = int(np.floor(box[0] / h)) - 1, int(np.ceil(box[1] / h)) + 1
    j0, j1 = int(np.floor(box[2] / h)) - 1, int(np.ceil(box[3] / h)) + 1
    s = (np.arange(sub) + 0.5) / sub
    fr = []
    for i in range(i0, i1):
        for j in range(j0, j1):
            x = (i + s[:, None]) * h + 0 * s[None, :]
            y = (j + s[None, :]) * h + 0 * s[:, None]
            fr.append(np.mean(footprint_inside(x.ravel(), y.ravel())))
    return np.array(fr)


def gated_pmf(n, p, kmax=None):
    """P(c = k), k = 0..kmax, of the gated approximation for n trials (real) and
    success probability p."""
    if n <= 0 or p <= 0:
        return np.array([1.0])
    pg = 1.0 if p >= 1 else -np.expm1(n * np.log1p(-p))
    m = max(n - 1.0, 0.0)
    mu, sg = m * p, np.sqrt(m * p * (1.0 - p))
    if kmax is None:
        kmax = int(np.ceil(mu + 12 * sg + 4))
    pmf = np.zeros(kmax + 1)
    pmf[0] = 1.0 - pg
    if sg == 0.0:
        pmf[1] = pg                              # x = 1 + mu exactly, mu < 1 when m = 0
        if 1.0 + mu >= 2.0:                      # only when p == 1 and n > 2
            pmf[1] = 0.0
            pmf[int(np.floor(1.0 + mu))] = pg
        return pmf
    # c = 1 <=> 1 + mu + sg z < 2 ; c = k >= 2 <=> k <= 1 + mu + sg z < k + 1
    pmf[1] = pg * norm.cdf((1.0 - mu) / sg)
    k = np.arange(2, kmax + 1)
    pmf[2:] = pg * (norm.cdf((k - mu) / sg) - norm.cdf((k - 1.0 - mu) / sg))
    return pmf


def gated_moments(n, p):
    pmf = gated_pmf(n, p)
    k = np.arange(pmf.size)
    mean = float(np.sum(k * pmf))
    var = float(np.sum(k * k * pmf) - mean * mean)
    return mean, var
