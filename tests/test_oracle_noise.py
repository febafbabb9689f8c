"""Pins of the noise and projection oracle (oracle/noise.py).

Expected values come from the published known-answer vectors of Philox4x32-10
(tests/golden), SciPy's Poisson distribution (quantile function and pmf),
moments fixed by the Poisson law, the flood height of Eq. 5, and
Beer-Lambert on a single energy.  Sec. II.G: noise is a Poisson scaling of
the counts on the detector; projections come back through the flood field.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import noise as nz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        ctr = [int(x, 16) for x in case["counter"]]
        key = [int(x, 16) for x in case["key"]]
        assert nz.philox4x32_10(ctr, key) == [int(x, 16) for x in case["out"]]


def test_uniform_pairs_order_and_range():
    seed = 0x0123456789ABCDEF
    pairs = nz.UniformPairs(7, 3, 11, seed)
    got = [pairs.next() for _ in range(4)]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    w0 = nz.philox4x32_10([7, 3, 11, 0], key)
    w1 = nz.philox4x32_10([7, 3, 11, 1], key)
    words = w0 + w1
    assert got == [((words[2 * i] + 0.5) / 2 ** 32, (words[2 * i + 1] + 0.5) / 2 ** 32) for i in range(4)]
    assert nz.uniform01(0) > 0.0 and nz.uniform01(0xFFFFFFFF) < 1.0


@pytest.mark.parametrize("lam", [0.3, 2.5, 9.0, 15.99])
def test_inversion_is_the_quantile(lam):
    # below the PTRS range the variate is F^-1(u) of the first uniform
    seed = 99
    for p in range(300):
        w = nz.philox4x32_10([p, 0, 0, 0], [seed, 0])
        u = nz.uniform01(w[0])
        k = nz.poisson(lam, nz.UniformPairs(p, 0, 0, seed))
        assert k == int(scipy.stats.poisson.ppf(u, lam)), (p, u)


def _draws(lam, n, seed, g=0):
    return np.array([nz.poisson(lam, nz.UniformPairs(p, g, 5, seed)) for p in range(n)])


@pytest.mark.parametrize("lam,n", [(16.0, 100000), (37.5, 40000), (1000.0, 40000), (2.5e5, 40000)])
def test_ptrs_distribution(lam, n):
    k = _draws(lam, n, seed=2024)
    # moments: mean lam, variance lam (Var of the sample variance ~ (lam + 2 lam^2) / n)
    z_mean = (k.mean() - lam) / math.sqrt(lam / n)
    z_var = (k.var(ddof=1) - lam) / math.sqrt((lam + 2 * lam * lam) / n)
    assert abs(z_mean) < 4.5 and abs(z_var) < 4.5, (z_mean, z_var)
    # chi-square against the Poisson pmf, bins merged to >= 50 expected counts
    lo, hi = int(scipy.stats.poisson.ppf(1e-6, lam)), int(scipy.stats.poisson.isf(1e-6, lam)) + 1
    edges = [lo]
    acc = 0.0
    for j in range(lo, hi):
        acc += scipy.stats.poisson.pmf(j, lam) * n
        if acc >= 50.0:
            edges.append(j + 1)
            acc = 0.0
    edges[-1] = hi
    cdf = scipy.stats.poisson.cdf(np.array(edges) - 1, lam)
    expected = np.diff(cdf) * n
    expected[0] += scipy.stats.poisson.cdf(lo - 1, lam) * n
    expected[-1] += scipy.stats.poisson.sf(hi - 1, lam) * n
    observed = np.histogram(np.clip(k, lo, hi - 1), bins=edges)[0]
    chi2 = float(((observed - expected) ** 2 / expected).sum())
    pval = scipy.stats.chi2.sf(chi2, len(expected) - 1)
    assert pval > 1e-4, (chi2, len(expected), pval)


def test_degenerate_means():
    pairs = nz.UniformPairs(0, 0, 0, 1)
    assert nz.poisson(0.0, pairs) == 0
    assert nz.poisson(-3.0, pairs) == 0
    assert nz.poisson(float("nan"), pairs) == 0


def _spectrum():
    rng = np.random.default_rng(5)
    E, G = 40, 4
    phi = rng.uniform(0.1, 1.0, E).astype(np.float32)
    eta = rng.uniform(0.2, 0.9, E).astype(np.float32)
    grp = (np.arange(E) * G) // E
    return phi, eta, grp, G


def test_count_scale_gives_the_flood_height():
    # Eq. 5: the open (I0 = 1) pixel holds H counts; group g gets the fluence share Phi_g / Phi
    phi, eta, grp, G = _spectrum()
    H = 3.0e4
    c = nz.count_scale(phi, eta, grp, G, H)
    p64, e64 = phi.astype(np.float64), eta.astype(np.float64)
    Wg = np.array([(p64 * e64)[grp == g].sum() for g in range(G)])
    share = np.array([p64[grp == g].sum() for g in range(G)]) / p64.sum()
    lam_open = c.astype(np.float64) * Wg
    np.testing.assert_allclose(lam_open, H * share, rtol=1e-6)
    assert abs(lam_open.sum() - H) < 1e-6 * H
    # a group without response gets no counts and passes unchanged
    eta0 = eta.copy()
    eta0[grp == 1] = 0.0
    c0 = nz.count_scale(phi, eta0, grp, G, H)
    assert c0[1] == 0.0 and np.all(c0[[0, 2, 3]] > 0)
    Y = np.full((1, G, 3), 0.25, np.float32)
    out = nz.noisy_signal(Y, c0, seed=3)
    np.testing.assert_array_equal(out[0, 1], Y[0, 1].astype(np.float64))


def test_noisy_signal_is_counts_over_scale():
    Y = np.array([[[0.0, 1e-3, 0.5], [2.0, 0.1, 7.0]]], np.float32)
    c = np.array([40.0, 1234.5], np.float32)
    n = nz.noisy_counts(Y, c, seed=77, a0=3)
    assert n[0, 0, 0] == 0
    out = nz.noisy_signal(Y, c, seed=77, a0=3)
    np.testing.assert_array_equal(out * c.astype(np.float64)[None, :, None], n.astype(np.float64))


def test_log_identity_single_energy(orc):
    # one energy, no scatter, unit spread: -ln(out / flood) is the line integral mu . L
    rng = np.random.default_rng(11)
    M = 3
    L = rng.uniform(0.0, 40.0, (1, 5, 6, M))
    mu = rng.uniform(0.005, 0.05, (M, 1))
    phi, eta = np.array([0.7]), np.array([0.4])
    i0 = rng.uniform(0.5, 2.0, (5, 6))
    Y = orc.spectral(L, mu, phi, eta, [0], 1, i0=i0).reshape(1, 1, 5, 6)
    K = np.ones((1, 1, 1))
    out = orc.psf(Y, K)
    Wg = np.array([0.7 * 0.4])
    flood = orc.psf(nz.flood_groups(Wg, i0, 5, 6), K)[0]
    p = nz.projection(out, flood)
    np.testing.assert_allclose(p[0], (L[0] @ mu)[..., 0], rtol=1e-12, atol=1e-12)


def test_object_free_flood_projects_to_zero(orc):
    # the flood of the projection equals the Eq. 3 signal of an empty ray through the same spread
    phi, eta, grp, G = _spectrum()
    rng = np.random.default_rng(8)
    nv, nu = 9, 12
    mu = rng.uniform(0.01, 0.1, (2, phi.size))
    i0 = rng.uniform(0.8, 1.2, (nv, nu))
    L = np.zeros((1, nv, nu, 2))
    Y = orc.spectral(L, mu, phi, eta, grp, G, i0=i0).reshape(G, 1, nv, nu).transpose(1, 0, 2, 3)
    K = rng.uniform(0.0, 1.0, (G, 5, 5))
    K /= K.sum(axis=(1, 2), keepdims=True)
    out = orc.psf(Y, K)
    Wg = np.array([(phi.astype(np.float64) * eta)[grp == g].sum() for g in range(G)])
    flood = orc.psf(nz.flood_groups(Wg, i0, nv, nu), K)[0]
    np.testing.assert_allclose(nz.projection(out, flood), 0.0, atol=1e-13)


def test_projection_floor():
    flood = np.array([[2.0, 4.0]])
    p = nz.projection(np.array([[[0.0, -1.0]]]), flood, floor=0.5)
    np.testing.assert_allclose(p, [[[math.log(4.0), math.log(8.0)]]])
    assert np.isinf(nz.projection(np.array([[[0.0]]]), np.array([[1.0]]))).all()


def test_noisy_projection_moments():
    # open beam times transmission T, single group: projection -ln(n / (c W)) has
    # mean p + 1 / (2 lam) and variance 1 / lam to first order (lam = H T)
    phi = np.array([1.0], np.float32)
    eta = np.array([0.5], np.float32)
    H = 2.0e4
    c = nz.count_scale(phi, eta, [0], 1, H)
    T = 0.3
    Y = np.full((1, 1, 8000), 0.5 * T, np.float32)
    noisy = nz.noisy_signal(Y, c, seed=4242)
    p = nz.projection(noisy[:, 0], np.array([0.5]))
    lam = H * T
    n = p.size
    z_mean = (p.mean() - (-math.log(T) + 0.5 / lam)) / math.sqrt(1.0 / (lam * n))
    z_var = (p.var(ddof=1) - 1.0 / lam) / (math.sqrt(2.0 / n) / lam)
    assert abs(z_mean) < 4.5 and abs(z_var) < 4.5, (z_mean, z_var)
