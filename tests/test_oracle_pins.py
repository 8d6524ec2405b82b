"""Pins of the FP64 oracle to the paper and to mathematics (CPU only).

Each test checks the oracle against something other than itself: a library
routine, a closed form, an invariant, quadrature, or brute force.  A plausible
mistake in the oracle (a dropped term, a wrong sign, index or operand order)
breaks at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtri as sp_ndtri

import oracle
from paper_2306_05051_amd import scenes
from oracle import bruteforce as bf


# ---------------------------------------------------------------------------
# Footprint (Sec. 5.1): axes of the pixel ellipse vs numpy's SVD
# ---------------------------------------------------------------------------
def test_footprint_matches_svd():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        J = rng.normal(size=(2, 2)) * 10.0 ** rng.uniform(-6, 0)
        res = oracle.footprint(J[0, 0], J[1, 0], J[0, 1], J[1, 1])
        U, S, Vt = np.linalg.svd(J)
        P, r, phi, s0 = res
        assert P == pytest.approx(abs(np.linalg.det(J)), rel=1e-10)
        assert s0 == pytest.approx(S[0], rel=1e-10)
        assert r == pytest.approx(max(S[0] / S[1], 1.0), rel=1e-8)
        e0 = U[:, 0]
        ref = math.atan2(e0[1], e0[0]) % math.pi
        d = abs(phi - ref)
        d = min(d, math.pi - d)
        cond = (S[0] + S[1]) / max(S[0] - S[1], 1e-300)
        assert d < 1e-9 * cond + 1e-12
        assert 0.0 <= phi < math.pi


def test_footprint_special_cases():
    # isotropic, axis aligned: ratio 1, orientation 0
    P, r, phi, s0 = oracle.footprint(0.5, 0.0, 0.0, 0.5)
    assert (P, r, phi, s0) == (0.25, 1.0, 0.0, 0.5)
    # stretched along v: major axis at pi/2
    P, r, phi, s0 = oracle.footprint(0.25, 0.0, 0.0, 1.0)
    assert P == 0.25 and r == 4.0 and phi == pytest.approx(math.pi / 2)
    assert oracle.footprint(1.0, 2.0, 2.0, 4.0) is None     # det J = 0


# ---------------------------------------------------------------------------
# Inverse normal CDF vs scipy; the 2^23 uniforms used by the method
# ---------------------------------------------------------------------------
def test_ndtri_matches_scipy():
    ks = np.unique(np.concatenate([np.arange(0, 64), 2**23 - 1 - np.arange(0, 64),
                                   np.random.default_rng(2).integers(0, 2**23, 4000)]))
    for k in ks:
        q = (2.0 * k + 1.0) * 2.0**-24
        z, ref = oracle.ndtri(q), sp_ndtri(q)
        assert abs(z - ref) <= 2e-14 * max(1.0, abs(ref)), (q, z, ref)


# ---------------------------------------------------------------------------
# Microfacet NDFs (Eq. 4): projected-area normalisation by quadrature;
# Smith Lambda: int D(m) <w,m>+ dm = (1 + Lambda(w)) <w,n>
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0])
def test_ndf_normalisation(kind, alpha):
    # substitution t = tan(theta) spreads the nodes over the lobe
    from scipy.integrate import quad
    f = lambda th: oracle.ndf(kind, alpha, math.cos(th)) * math.cos(th) * math.sin(th) * 2 * math.pi
    val = quad(f, 0, math.pi / 2, points=[math.atan(alpha)], limit=400, epsabs=1e-13, epsrel=1e-11)[0]
    assert val == pytest.approx(1.0, rel=2e-7)


@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0])
def test_ndf_textbook_closed_forms(alpha):
    """Sec. 3 names the standard NDFs GGX and Beckmann; their textbook forms
    (Walter et al. 2007) in the half-angle theta_m:
    GGX D = alpha^2 / (pi cos^4 (alpha^2 + tan^2)^2),
    Beckmann D = exp(-tan^2 / alpha^2) / (pi alpha^2 cos^4).
    Normalisation alone holds for any consistent roughness convention; this
    fixes the convention (alpha, not alpha^2, is the roughness)."""
    for th in np.linspace(0.0, 1.45, 30):
        c, t2 = math.cos(th), math.tan(th) ** 2
        ggx = alpha**2 / (math.pi * c**4 * (alpha**2 + t2) ** 2)
        beck = math.exp(-t2 / alpha**2) / (math.pi * alpha**2 * c**4)
        assert oracle.ndf(0, alpha, c) == pytest.approx(ggx, rel=1e-12, abs=1e-300)
        assert oracle.ndf(1, alpha, c) == pytest.approx(beck, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("alpha", [0.1, 0.4, 0.9])
@pytest.mark.parametrize("theta_deg", [20.0, 60.0, 80.0])
def test_smith_lambda_identity(kind, alpha, theta_deg):
    th = math.radians(theta_deg)
    w = np.array([math.sin(th), 0.0, math.cos(th)])
    nt, npp = 700, 720
    # Gauss-Legendre in theta_m (in tan space) and midpoint in phi_m
    x, wx = np.polynomial.legendre.leggauss(nt)
    thm = 0.5 * (x + 1) * (math.pi / 2)
    wth = wx * (math.pi / 4)
    ph = (np.arange(npp) + 0.5) * (2 * math.pi / npp)
    TH, PH = np.meshgrid(thm, ph, indexing="ij")
    M = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    D = np.vectorize(lambda c: oracle.ndf(kind, alpha, c))(np.cos(TH))
    proj = np.maximum(M @ w, 0.0)
    integ = np.sum(D * proj * np.sin(TH) * wth[:, None]) * (2 * math.pi / npp)
    lam = oracle.smith_lambda(kind, alpha, math.cos(th))
    assert integ == pytest.approx((1.0 + lam) * math.cos(th), rel=5e-4)


# ---------------------------------------------------------------------------
# Gated binomial (Eqs. 16-18)
# ---------------------------------------------------------------------------
def _grid_thetas(n):
    k = (np.arange(n) * (2**23 // n)) + (2**23 // n) // 2
    return (2.0 * k + 1.0) * 2.0**-24


def test_gate_probability_is_one_minus_q_pow_n():
    th = _grid_thetas(1 << 16)
    for n, p in [(1.0, 0.3), (2.0, 0.1), (7.5, 0.02), (40.0, 0.05), (0.4, 0.5)]:
        opened = np.array([oracle.gated_count(n, p, t0, 0.5) > 0 for t0 in th])
        assert opened.mean() == pytest.approx(1.0 - (1.0 - p) ** n, abs=2.0 / th.size)


def test_one_trial_is_bernoulli():
    th = _grid_thetas(1 << 14)
    for p in (0.05, 0.5, 0.9):
        c = np.array([[oracle.gated_count(1.0, p, t0, t1) for t1 in th[::512]] for t0 in th[::64]])
        assert set(np.unique(c)) <= {0.0, 1.0}
        assert c.mean() == pytest.approx(p, abs=2.0 / 256)


@pytest.mark.parametrize("n,p", [(2.0, 0.1), (6.0, 0.3), (30.0, 0.2), (200.0, 0.05), (3.3, 0.7)])
def test_gated_pmf_closed_form(n, p):
    """Realised histogram over a dense theta1 grid (gate forced open) against the
    closed form through Phi."""
    th1 = _grid_thetas(1 << 16)
    c = np.array([oracle.gated_count(n, p, 0.0, t1) for t1 in th1]).astype(int)
    pmf = bf.gated_pmf(n, p)
    pg = pmf[1:].sum()
    hist = np.bincount(c, minlength=pmf.size)[: pmf.size] / c.size
    # conditional on an open gate
    assert np.all(c >= 1)
    assert np.max(np.abs(hist[1:] - pmf[1:] / pg)) < 3.0 / th1.size + 1e-9


@pytest.mark.parametrize("n,p", [(6.0, 0.3), (30.0, 0.2), (3.3, 0.7)])
def test_gated_count_histogram_from_hashed_uniforms(n, p):
    """The whole chain of one texel's count: gate and count uniforms hashed
    from texel keys and the slot-0 / slot-1 angular keys (H(prefix, angular
    key), theta = (2 (h >> 9) + 1) 2^-24), then the gated binomial.  The
    realised histogram over 60000 texels, zeros included, against the closed
    form through Phi (chi-squared)."""
    from scipy import stats
    ang = [oracle.hash_step(0x13198A2E, (5 + 16384) | ((7 + 16384) << 15) | (s << 30)) for s in (0, 1)]
    root = oracle.hash_step(0x243F6A88, 11)
    c = np.empty(60000, np.int64)
    k = 0
    for i in range(300):
        hi = oracle.hash_step(root, i)
        for j in range(200):
            pre = oracle.hash_step(hi, j)
            th0, th1 = [((oracle.hash_step(pre, a) >> 9) * 2 + 1) / 2.0**24 for a in ang]
            c[k] = int(oracle.gated_count(n, p, th0, th1))
            k += 1
    pmf = bf.gated_pmf(n, p)
    obs = np.bincount(c, minlength=pmf.size)
    assert obs.size == pmf.size, "count beyond the closed form's support"
    exp = pmf * c.size
    keep = exp >= 5.0
    chi2 = float(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])) + \
        float((obs[~keep].sum() - exp[~keep].sum()) ** 2 / max(exp[~keep].sum(), 1.0))
    dof = int(keep.sum())
    assert stats.chi2.sf(chi2, dof) > 1e-4, (obs, exp)


# ---------------------------------------------------------------------------
# Hash: uniformity and independence of the per-texel uniforms
# ---------------------------------------------------------------------------
def test_hash_avalanche():
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(300):
        h, w = int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))
        base = oracle.hash_step(h, w)
        for b in range(32):
            flips.append(bin(base ^ oracle.hash_step(h, w ^ (1 << b))).count("1"))
            flips.append(bin(base ^ oracle.hash_step(h ^ (1 << b), w)).count("1"))
    assert np.mean(flips) == pytest.approx(16.0, abs=0.15)


def test_hash_uniform_and_independent_on_texel_keys():
    # neighbouring texels of one grid and neighbouring angular cells
    vals = np.array([oracle.hash_step(oracle.hash_step(oracle.hash_step(0x1234, i), j), a)
                     for i in range(64) for j in range(64) for a in range(4)], dtype=np.uint64)
    u = ((vals >> 9) * 2 + 1) / 2.0**24
    hist = np.bincount((u * 64).astype(int), minlength=64)
    chi2 = np.sum((hist - u.size / 64) ** 2 / (u.size / 64))
    assert chi2 < 120.0                       # 63 dof, p ~ 1e-5 cut
    g = u.reshape(64, 64, 4)
    for a, b in [(g[1:, :, 0], g[:-1, :, 0]), (g[:, 1:, 0], g[:, :-1, 0]), (g[..., 1], g[..., 0])]:
        assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 0.05


# ---------------------------------------------------------------------------
# Random-number table variant (Sec. 6.3: the two uniforms of a gated binomial
# read from a small precomputed texture)
# ---------------------------------------------------------------------------
def test_rng_table_entries_uniform_and_uncorrelated():
    t = np.array([oracle.rng_table_entry(0x5EED, i) for i in range(1 << 14)], dtype=np.uint64)
    u = ((t >> 9) * 2 + 1) / 2.0**24
    hist = np.bincount((u * 64).astype(int), minlength=64)
    chi2 = np.sum((hist - u.size / 64) ** 2 / (u.size / 64))
    assert chi2 < 120.0                       # 63 dof
    assert abs(np.corrcoef(u[1:], u[:-1])[0, 1]) < 0.05
    assert len(np.unique(t)) > 0.999 * t.size
    other = np.array([oracle.rng_table_entry(0x5EEE, i) for i in range(1 << 10)], dtype=np.uint64)
    assert abs(np.corrcoef(u[: 1 << 10], ((other >> 9) * 2 + 1) / 2.0**24)[0, 1]) < 0.1


def _murmur3_x86_32(data, seed):
    """MurmurHash3_x86_32 (Appleby): 4-byte little-endian blocks mixed with
    k *= c1, rotl 15, k *= c2 into h (h ^= k, rotl 13, h = 5 h + n), the tail
    bytes mixed the same way without the h steps, h ^= length, and the
    finaliser, which here is the oracle's."""
    m32 = 0xFFFFFFFF
    c1, c2 = 0xCC9E2D51, 0x1B873593

    def rotl(x, r):
        return ((x << r) | (x >> (32 - r))) & m32

    def mix(k):
        return (rotl((k * c1) & m32, 15) * c2) & m32

    h, nb = seed, len(data) // 4
    for i in range(nb):
        h = rotl(h ^ mix(int.from_bytes(data[4 * i:4 * i + 4], "little")), 13)
        h = (h * 5 + 0xE6546B64) & m32
    tail = data[4 * nb:]
    if tail:
        h ^= mix(int.from_bytes(tail, "little"))
    return oracle.fmix32(h ^ len(data))


def test_fmix32_is_the_murmur3_finaliser():
    """The oracle's fmix32 against MurmurHash3_x86_32's published test vectors
    (tests/golden/murmur3_x86_32_vectors.txt): the empty-input ones are
    fmix32(seed) exactly; a wrong shift, multiplier or step order fails them."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "murmur3_x86_32_vectors.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 13
    for data, seed, want in rows:
        b = b"" if data == "-" else bytes.fromhex(data)
        assert _murmur3_x86_32(b, int(seed, 16)) == int(want, 16), (data, seed)
        if data == "-":
            assert oracle.fmix32(int(seed, 16)) == int(want, 16)


def _table_scene():
    gb, mats, lights = scenes.four_k(48, 24, seed=13, n_mat=3, n_light=2)
    return gb, mats, lights


def test_rng_table_full_width_is_the_hash():
    """A table of 2^32 words with seed 0 holds H(0, i) = fmix32(i + c) at index
    i, so reading it at index texel key XOR angular key gives H(texel key,
    angular key): the table mode must then reproduce the hash mode bit for bit
    (every debug plane, every count, the radiance)."""
    gb, mats, lights = _table_scene()
    ref, dr = oracle.shade(gb, mats, lights, debug=True)
    out, dt = oracle.shade(gb, mats, lights, debug=True, rng_table=(32, 0))
    assert int(dr["n_open"].sum()) > 20
    np.testing.assert_array_equal(out, ref)
    for k in dr:
        np.testing.assert_array_equal(dt[k], dr[k], err_msg=k)
    # a partial table or another seed changes the words, not the geometry
    _, d12 = oracle.shade(gb, mats, lights, debug=True, rng_table=(12, 0))
    _, ds = oracle.shade(gb, mats, lights, debug=True, rng_table=(32, 1))
    for d in (d12, ds):
        assert not np.array_equal(d["theta_sum"], dr["theta_sum"])
        for k in ("flags", "n_probe", "level", "cell", "key_sum", "akey_sum", "n_gate", "n_live"):
            np.testing.assert_array_equal(d[k], dr[k], err_msg=k)


def test_rng_table_small_table_repeats_words():
    """With 2^1 words every gate word is one of two table entries: theta_sum
    of a pixel is a combination of the two with n_gate terms."""
    gb, mats, lights = _table_scene()
    _, d = oracle.shade(gb, mats, lights, debug=True, rng_table=(1, 7))
    t0, t1 = oracle.rng_table_entry(7, 0), oracle.rng_table_entry(7, 1)
    ng = d["n_gate"].astype(np.int64)
    ts = d["theta_sum"].astype(np.int64)
    ok = ng > 0
    # theta_sum = a t0 + (n_gate - a) t1 (mod 2^32) for some 0 <= a <= n_gate
    found = np.zeros(ng.shape, bool)
    for a in range(int(ng.max()) + 1):
        found |= ((a * t0 + (ng - a) * t1 - ts) % (1 << 32) == 0) & (a <= ng)
    assert ok.sum() > 100 and np.all(found[ok])


# ---------------------------------------------------------------------------
# Grid family: distributed weights (Eq. 10, Sec. 5.2, Sec. 6.1)
# ---------------------------------------------------------------------------
def _cell_uv(rk, phi, K):
    rho = min(max(math.log2(rk), 0.0), K)
    kap = min(int(math.floor(rho)), K - 1)
    M = 2 ** (kap + 1)
    q = phi / (math.pi / M)
    j = min(int(math.floor(q)), M - 1)
    return kap, j, rho - kap, q - j, M


def test_area_conservation_and_weights():
    rng = np.random.default_rng(4)
    for _ in range(4000):
        Pk = 10.0 ** rng.uniform(-12, 1)
        rk = 2.0 ** rng.uniform(0, 4)
        phi = rng.uniform(0, math.pi)
        nodes, cell, _ = oracle.grid_nodes(Pk, rk, phi, 4)
        w = np.array([n[3] for n in nodes])
        assert len(nodes) <= 4 and np.all(w >= 0)
        assert w.sum() == pytest.approx(1.0, abs=1e-13)
        area = sum(n[3] * 2.0 ** n[0] for n in nodes)
        assert area == pytest.approx(Pk, rel=1e-13)
        l = cell["level"]
        assert 2.0 ** l <= Pk < 2.0 ** (l + 1)
        assert {n[0] for n in nodes} <= {l, l + 1}


def test_tetra_barycentric_reconstruction():
    """For cells away from ring 0 the weights are barycentric coordinates of the
    point (u, t, s) in the cell's (ratio, orientation, scale) coordinates."""
    rng = np.random.default_rng(5)
    for _ in range(3000):
        Pk = 10.0 ** rng.uniform(-9, -3)
        rk = 2.0 ** rng.uniform(1.0, 4.0)
        phi = rng.uniform(0, math.pi)
        kap, j, u, t, M = _cell_uv(rk, phi, 4)
        nodes, cell, _ = oracle.grid_nodes(Pk, rk, phi, 4)
        l = cell["level"]
        ts = Pk / 2.0**l - 1.0
        pos = np.zeros(3)
        for (nl, nk, nm, w) in nodes:
            if nk == kap:
                tt = (nm - j) % M            # 0 or 1
                uu = 0.0
            else:
                assert nk == kap + 1
                tt = ((nm - 2 * j) % (2 * M)) / 2.0
                uu = 1.0
            assert tt in (0.0, 0.5, 1.0)
            pos += w * np.array([uu, tt, nl - l])
        assert np.allclose(pos, [u, t, ts], atol=1e-12), (pos, u, t, ts)


def test_isotropic_reductions():
    # r = 1: only the isotropic grid (ratio level 0) carries weight (the
    # two-level law of Sec. 4.2); K = 0: isotropic family only.
    rng = np.random.default_rng(6)
    for _ in range(500):
        Pk, phi = 10.0 ** rng.uniform(-9, -3), rng.uniform(0, math.pi)
        nodes, _, _ = oracle.grid_nodes(Pk, 1.0, phi, 4)
        assert all(n[1] == 0 for n in nodes if n[3] > 0)
        nodes, _, _ = oracle.grid_nodes(Pk, 8.0, phi, 0)
        assert len(nodes) == 2 and all(n[1] == 0 and n[2] == 0 for n in nodes)
        ts = Pk / 2.0 ** nodes[0][0] - 1.0
        assert nodes[1][3] == pytest.approx(ts, abs=1e-15)  # Eq. 10 weight of the top level
    # exact power of two and r = 1: a single grid
    nodes, _, _ = oracle.grid_nodes(2.0**-10, 1.0, 0.3, 4)
    assert [n for n in nodes if n[3] > 0] == [(-10, 0, 0, 1.0)]


def _wmap(nodes):
    out = {}
    for (l, k, m, w) in nodes:
        out[(l, k, m)] = out.get((l, k, m), 0.0) + w
    return out


def _wdist(a, b):
    keys = set(a) | set(b)
    return max(abs(a.get(k, 0.0) - b.get(k, 0.0)) for k in keys)


def test_weights_continuous_across_cells():
    """Coherence between consecutive LODs, ratios and orientations: the weight
    of each grid is continuous (Sec. 1: coherence between consecutive LODs)."""
    eps = 1e-9
    rng = np.random.default_rng(7)
    for _ in range(300):
        phi = rng.uniform(0.01, math.pi - 0.01)
        rk = 2.0 ** rng.uniform(0.1, 3.9)
        l = int(rng.integers(-30, -5))
        Pb = 2.0**l
        a = _wmap(oracle.grid_nodes(Pb * (1 - eps), rk, phi)[0])
        b = _wmap(oracle.grid_nodes(Pb * (1 + eps), rk, phi)[0])
        assert _wdist(a, b) < 1e-7
        kb = int(rng.integers(1, 4))
        a = _wmap(oracle.grid_nodes(3e-7, 2.0 ** (kb - eps), phi)[0])
        b = _wmap(oracle.grid_nodes(3e-7, 2.0 ** (kb + eps), phi)[0])
        assert _wdist(a, b) < 1e-7
        kap = int(rng.integers(0, 4))
        M = 2 ** (kap + 1)
        jb = int(rng.integers(1, M))
        rr = 2.0 ** (kap + rng.uniform(0.05, 0.95))
        a = _wmap(oracle.grid_nodes(3e-7, rr, jb * math.pi / M - eps)[0])
        b = _wmap(oracle.grid_nodes(3e-7, rr, jb * math.pi / M + eps)[0])
        assert _wdist(a, b) < 1e-7
    # orientation wraps at pi: 0+ and pi- select the same grids
    a = _wmap(oracle.grid_nodes(3e-7, 5.0, eps)[0])
    b = _wmap(oracle.grid_nodes(3e-7, 5.0, math.pi - eps)[0])
    assert _wdist(a, b) < 1e-7


# ---------------------------------------------------------------------------
# Simplex lattice (Sec. 6.2): barycentric reconstruction of the point
# ---------------------------------------------------------------------------
def test_simplex_reconstruction():
    rng = np.random.default_rng(8)
    for _ in range(3000):
        l, k = int(rng.integers(-30, -5)), int(rng.integers(0, 5))
        m = int(rng.integers(0, 2 ** (k + 1))) if k > 0 else 0
        cx, cy = rng.uniform(-2, 2, 2)
        verts, beta, _ = oracle.simplex(cx, cy, l, k, m)
        beta = np.array(beta)
        assert np.all(beta >= 0) and beta.sum() == pytest.approx(1.0, abs=1e-12)
        # lattice vertex (i, j) sits at ((i - j/2) wx, j wy) in the grid frame,
        # rotated back by +phi_g into uv space
        phig = m * math.pi / 2 ** (k + 1) if k > 0 else 0.0
        wx, wy = math.sqrt(2.0 ** (l + k)), math.sqrt(2.0 ** (l - k))
        pts = []
        for (i, j) in verts:
            gx, gy = (i - 0.5 * j) * wx, j * wy
            pts.append((math.cos(phig) * gx - math.sin(phig) * gy, math.sin(phig) * gx + math.cos(phig) * gy))
        rec = beta @ np.array(pts)
        scale = max(abs(cx), abs(cy), 1.0)
        assert np.allclose(rec, [cx, cy], atol=1e-12 * scale / min(wx, wy) * wx), (rec, cx, cy)
        # the three vertices form a triangle of area A/2 (cell area A = 2^l)
        (x0, y0), (x1, y1), (x2, y2) = pts
        tri = 0.5 * abs((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))
        assert tri == pytest.approx(0.5 * 2.0**l, rel=1e-9)


def test_tangent_frame_orthonormal_right_handed():
    """The frame that indexes the angular grid (Duff et al.'s branchless ONB,
    a choice) must be an orthonormal right-handed basis with n as third axis,
    so that the projected half vector (<h,t>, <h,b>) keeps |.|^2 = 1 - <h,n>^2
    and h = n lands on the grid origin."""
    rng = np.random.default_rng(5)
    ns = rng.normal(size=(3000, 3))
    ns = np.concatenate([ns, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 1e-12], [1e-9, 0, -1],
                              [0.3, -0.2, -1e-15]]])
    ns /= np.linalg.norm(ns, axis=1, keepdims=True)
    for n in ns:
        t, b = (np.array(x) for x in oracle.tangent_frame(n))
        M = np.stack([t, b, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12), n
        assert np.allclose(np.cross(t, b), n, atol=1e-12), n
        h = rng.normal(size=3)
        h /= np.linalg.norm(h)
        assert np.dot(h, t) ** 2 + np.dot(h, b) ** 2 == pytest.approx(1.0 - np.dot(h, n) ** 2, abs=1e-12)


def test_probe_centres_partition_the_major_axis():
    """Sec. 4.2 with reading S25: the n_pr sub-footprints of an over-long
    footprint sit on its major axis (the leading singular vector of J) and
    split the ellipse's major-axis extent [-sigma0/2, sigma0/2] into equal,
    contiguous segments centred on the pixel."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        J = rng.normal(size=(2, 2)) * 10.0 ** rng.uniform(-4, -1)
        fp = oracle.footprint(J[0, 0], J[1, 0], J[0, 1], J[1, 1])
        if fp is None:
            continue
        P, r, phi, s0 = fp
        U, S, Vt = np.linalg.svd(J)
        axis = np.array([math.cos(phi), math.sin(phi)])
        assert abs(abs(np.dot(axis, U[:, 0])) - 1.0) < 1e-9
        assert s0 == pytest.approx(S[0], rel=1e-12)
        u, v = rng.uniform(-3, 3, size=2)
        for n_pr in (1, 2, 3, 7, 21):
            c = np.array([oracle.probe_centre(u, v, phi, s0, n_pr, k) for k in range(n_pr)])
            d = (c - [u, v]) @ axis                          # along the major axis
            perp = (c - [u, v]) @ np.array([-axis[1], axis[0]])
            assert np.allclose(perp, 0.0, atol=1e-12 * (abs(u) + abs(v) + s0))
            assert np.mean(d) == pytest.approx(0.0, abs=1e-12 * (abs(u) + abs(v) + s0))
            lo, hi = d - s0 / (2 * n_pr), d + s0 / (2 * n_pr)
            assert lo[0] == pytest.approx(-s0 / 2, rel=1e-9) and hi[-1] == pytest.approx(s0 / 2, rel=1e-9)
            assert np.allclose(lo[1:], hi[:-1], rtol=0, atol=1e-9 * s0)
