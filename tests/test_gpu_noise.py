"""GPU parity of the noise and projection stage (Sec. II.G, Eq. 5) with the oracle.

* Count scale: both sides sum in FP64 in bin order, so the float32 values
  must be equal.
* Poisson draws: integer work, bit-exact.  Both sides take every decision in
  FP64 from the same float32 mean and the same Philox4x32-10 words; only the
  last bit of a transcendental (exp, log) may differ, which can move a draw
  only for a uniform within ~1e-16 of a decision boundary.
* Log conversion: FP32 on the GPU, the float32 ratio and logf each add at
  most an ulp, so |proj - ref| <= 3e-7 + 1e-6 |ref|.
* Flood profile and noiseless projections: FP32 against FP64, from the
  1e-5 relative bound of the detected profile (an absolute 2e-5 on -ln).
* Noisy projections: moments against the Poisson law, and independence of
  the draws from chunking.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
import synth
from oracle import noise as onz

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _spectral(fc, rng, E=40, G=4, uneven=True):
    phi = rng.uniform(0.1, 1.0, E).astype(np.float32)
    eta = rng.uniform(0.2, 0.9, E).astype(np.float32)
    if uneven:
        grp = np.sort(np.concatenate([np.arange(G), rng.integers(0, G, E - G)])).astype(np.int32)
    else:
        grp = ((np.arange(E) * G) // E).astype(np.int32)
    mu = rng.uniform(0.01, 0.1, (2, E)).astype(np.float32)
    sp = fc.Spectral(mu=_dev(mu), phi=_dev(phi), eta=_dev(eta), n_groups=G, group_of_bin=grp)
    return sp, phi, eta, grp


def test_count_scale_equals_oracle(fc):
    rng = np.random.default_rng(3)
    for H in (1.0, 3.7e4, 2.5e9):
        sp, phi, eta, grp = _spectral(fc, rng)
        got = fc.fcat_count_scale(sp, H).cpu().numpy()
        ref = onz.count_scale(phi, eta, grp, sp.n_groups, H)
        np.testing.assert_array_equal(got, ref)
    # a group without response
    sp, phi, eta, grp = _spectral(fc, rng, uneven=False)
    eta0 = eta.copy()
    eta0[grp == 2] = 0.0
    sp.eta = _dev(eta0)
    got = fc.fcat_count_scale(sp, 1e4).cpu().numpy()
    assert got[2] == 0.0
    np.testing.assert_array_equal(got, onz.count_scale(phi, eta0, grp, sp.n_groups, 1e4))


def _signals(rng, A, G, plane):
    """Group signals over six decades plus exact zeros; scales put the means
    in both sampler ranges (below and above 16)."""
    Y = np.exp(rng.uniform(np.log(1e-6), 0.0, (A, G, plane))).astype(np.float32)
    Y[rng.random((A, G, plane)) < 0.02] = 0.0
    scale = np.exp(rng.uniform(np.log(10.0), np.log(3e5), G)).astype(np.float32)
    return Y, scale


def test_poisson_bit_exact_small(fc):
    rng = np.random.default_rng(17)
    A, G, nv, nu = 3, 3, 29, 37                     # plane of 1073: four blocks and a ragged tail
    Y, scale = _signals(rng, A, G, nv * nu)
    scale[1] = 0.0                                  # a group that passes unchanged
    seed = 0xDEADBEEF12345678
    Yd = _dev(Y.reshape(A, G, nv, nu))
    fc.fcat_poisson(Yd, _dev(scale), seed, angle_base=5)
    got = Yd.cpu().numpy().reshape(A, G, nv * nu).astype(np.float64)
    n_ref = onz.noisy_counts(Y, scale, seed, a0=5)
    for g in range(G):
        if scale[g] > 0:
            n_got = np.rint(got[:, g] * np.float64(scale[g])).astype(np.int64)
            mism = np.argwhere(n_got != n_ref[:, g])
            assert mism.size == 0, (g, mism[:5], n_got[tuple(mism[0])], n_ref[:, g][tuple(mism[0])])
            np.testing.assert_allclose(got[:, g], n_ref[:, g] / np.float64(scale[g]), rtol=2 ** -23, atol=0)
        else:
            np.testing.assert_array_equal(got[:, g], Y[:, g])
    lam = scale[None, :, None].astype(np.float64) * Y
    assert (lam[lam > 0] < 16).sum() > 500 and (lam >= 16).sum() > 500


def test_poisson_bit_exact_hard_means(fc):
    # 120k draws concentrated where the kernel's single-precision pass is
    # closest to its limits: means just below and above 16, tiny means, means
    # of 1e5..1e7, and float32 means one ulp apart
    rng = np.random.default_rng(41)
    lam = np.concatenate([
        rng.uniform(15.0, 16.0, 20000), rng.uniform(16.0, 17.0, 20000),
        np.exp(rng.uniform(np.log(1e-4), np.log(1.0), 20000)),
        np.exp(rng.uniform(np.log(1e5), np.log(1.6e7), 20000)),
        np.nextafter(np.float32(23.5), np.float32(30.0)) * np.ones(20000),
        rng.uniform(16.0, 2000.0, 20000)]).astype(np.float32)
    P = lam.size
    Y = lam.reshape(1, 1, P)
    scale = np.ones(1, np.float32)
    Yd = _dev(Y)
    fc.fcat_poisson(Yd, _dev(scale), 0xC0FFEE, angle_base=3)
    got = np.rint(Yd.cpu().numpy().reshape(-1).astype(np.float64)).astype(np.int64)
    ref = onz.noisy_counts(Y, scale, 0xC0FFEE, a0=3).reshape(-1)
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, [(int(i), float(lam[i]), int(got[i]), int(ref[i])) for i in bad[:5]]


def test_poisson_independent_of_launch_split(fc):
    import torch
    rng = np.random.default_rng(5)
    A, G, plane = 6, 2, 700
    Y, scale = _signals(rng, A, G, plane)
    sc = _dev(scale)
    whole = _dev(Y)
    fc.fcat_poisson(whole, sc, 99, angle_base=10)
    parts = _dev(Y)
    for a in range(A):
        fc.fcat_poisson(parts[a:a + 1], sc, 99, angle_base=10 + a)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(whole.cpu().numpy(), parts.cpu().numpy())
    other = _dev(Y)
    fc.fcat_poisson(other, sc, 100, angle_base=10)
    assert (other.cpu().numpy() != whole.cpu().numpy()).mean() > 0.5


@pytest.mark.parametrize("lam", [0.7, 6.0, 15.9, 16.0, 45.0, 1.0e3, 2.0e5])
def test_poisson_distribution(fc, lam):
    # 2^20 draws of one mean: moments and chi-square against the Poisson pmf
    n = 1 << 20
    Y = _dev(np.full((1, 1, n), 1.0, np.float32))
    fc.fcat_poisson(Y, _dev(np.array([lam], np.float32)), 1234)
    k = np.rint(Y.cpu().numpy().reshape(-1) * np.float64(np.float32(lam))).astype(np.int64)
    lam32 = float(np.float32(lam))
    z_mean = (k.mean() - lam32) / math.sqrt(lam32 / n)
    z_var = (k.var(ddof=1) - lam32) / math.sqrt((lam32 + 2 * lam32 * lam32) / n)
    assert abs(z_mean) < 5 and abs(z_var) < 5, (z_mean, z_var)
    lo = int(scipy.stats.poisson.ppf(1e-7, lam32))
    hi = int(scipy.stats.poisson.isf(1e-7, lam32)) + 1
    edges = [lo]
    acc = 0.0
    for j in range(lo, hi):
        acc += scipy.stats.poisson.pmf(j, lam32) * n
        if acc >= 100.0:
            edges.append(j + 1)
            acc = 0.0
    edges[-1] = hi
    expected = np.diff(scipy.stats.poisson.cdf(np.array(edges) - 1, lam32)) * n
    expected[0] += scipy.stats.poisson.cdf(lo - 1, lam32) * n
    expected[-1] += scipy.stats.poisson.sf(hi - 1, lam32) * n
    observed = np.histogram(np.clip(k, lo, hi - 1), bins=edges)[0]
    chi2 = float(((observed - expected) ** 2 / expected).sum())
    assert scipy.stats.chi2.sf(chi2, len(expected) - 1) > 1e-5, chi2


def test_poisson_full_size_sampled(fc):
    # group signals of the contrast workload (360 angles, 8 groups, 64 x 1024)
    # in one call; 3000 sampled elements against the oracle, one by one
    import torch
    rng = np.random.default_rng(2011)
    A, G, plane = 360, 8, 64 * 1024
    Y = np.exp(rng.uniform(np.log(1e-5), 0.0, (A, G, plane)).astype(np.float32))
    scale = np.exp(rng.uniform(np.log(1e2), np.log(1e6), G)).astype(np.float32)
    Yd = _dev(Y)
    seed = 7
    fc.fcat_poisson(Yd, _dev(scale), seed, angle_base=0)
    torch.cuda.synchronize()
    idx = [(int(rng.integers(A)), int(rng.integers(G)), int(rng.integers(plane))) for _ in range(3000)]
    idx += [(A - 1, G - 1, plane - 1), (0, 0, 0)]
    sel = torch.tensor([(a * G + g) * plane + p for a, g, p in idx], device="cuda")
    got = Yd.reshape(-1)[sel].cpu().numpy().astype(np.float64)
    for (a, g, p), y in zip(idx, got):
        n_ref = onz.noisy_count(float(Y[a, g, p]), float(scale[g]), p, g, a, seed)
        assert int(np.rint(y * np.float64(scale[g]))) == n_ref, (a, g, p)


def test_log_projection_parity(fc):
    rng = np.random.default_rng(9)
    A, nv, nu = 4, 13, 300
    flood = rng.uniform(0.5, 2.0, (nv, nu)).astype(np.float32)
    out = (flood[None] * np.exp(-rng.uniform(0.0, 12.0, (A, nv, nu)))).astype(np.float32)
    out[0, 0, :5] = 0.0
    out[1, 1, :3] = -1e-3
    for floor in (0.0, 1e-4):
        got = fc.fcat_log_projection(_dev(out), _dev(flood), floor=floor).cpu().numpy()
        ref = onz.projection(out, flood, floor)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin) and np.all(got[~fin] == np.inf)
        np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-6, atol=3e-7)
    # in place
    od = _dev(out)
    fc.fcat_log_projection(od, _dev(flood), floor=1e-4, proj=od)
    np.testing.assert_allclose(od.cpu().numpy(), onz.projection(out, flood, 1e-4), rtol=1e-6, atol=3e-7)


def _every_term_config(rng):
    cfg = synth.make_config(1)
    g, s = cfg.geometry, cfg.spectral
    s.flood = rng.uniform(0.8, 1.2, size=(g.nv, g.nu)).astype(np.float32)
    s.n_groups = 3
    s.group_of_bin = np.array([0] * 5 + [1] * 20 + [2] * 7, np.int32)
    cfg.scatter = synth.scatter_blobs(rng, g.n_angles, g.nu, g.nv, (30, 60), (4, 8))
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 3, 15))
    return cfg


def _oracle_flood(cfg, use_psf=True):
    s, g = cfg.spectral, cfg.geometry
    p64, e64 = s.phi.astype(np.float64), s.eta.astype(np.float64)
    Wg = np.array([(p64 * e64)[s.group_of_bin == k].sum() for k in range(s.n_groups)])
    Yf = onz.flood_groups(Wg, s.flood, g.nv, g.nu)
    K = cfg.psf.kernels if (use_psf and cfg.psf is not None) else np.ones((s.n_groups, 1, 1))
    return oracle.psf(Yf, K)[0]


def test_flood_profile_parity(fc):
    from conftest import rel_err
    rng = np.random.default_rng(21)
    cfg = _every_term_config(rng)
    pb = fc.upload(cfg)
    for use_psf in (True, False):
        got = fc.fcat_flood_profile(pb.spectral, pb.psf if use_psf else None, cfg.geometry.nv,
                                    cfg.geometry.nu).cpu().numpy()
        assert rel_err(got, _oracle_flood(cfg, use_psf)).max() <= 1e-5


@pytest.mark.parametrize("mode", ["plain", "split_bf16"])
def test_noiseless_projections_parity(fc, mode):
    rng = np.random.default_rng(22)
    cfg = _every_term_config(rng)
    pb = fc.upload(cfg)
    got = fc.fcat_projections(pb, None, mode=mode).cpu().numpy()
    angles = list(range(0, 45, 4))
    ref = onz.projection(oracle.project(cfg, angles), _oracle_flood(cfg))
    tol = 2e-5 if mode == "plain" else 2e-3
    err = np.abs(got[angles] - ref)
    print(f"{mode}: max |proj - ref| {err.max():.3e}")
    assert err.max() <= tol


def test_noisy_projections_statistics(fc):
    # no spread: Var(out) = sum_g Y_g / c_g, so z = (noisy - noiseless) out / sqrt(sum_g Y_g / c_g)
    # is close to N(0, 1) over the pixels (delta method; lambda >= ~50 here)
    rng = np.random.default_rng(23)
    cfg = _every_term_config(rng)
    cfg.psf = None
    pb = fc.upload(cfg)
    H = 5.0e5
    noise = fc.Noise(counts_per_pixel=H, seed=31337)
    noisy = fc.fcat_projections(pb, noise).cpu().numpy()
    clean = fc.fcat_projections(pb, None).cpu().numpy()
    angles = list(range(0, 45, 3))
    out, Yg = oracle.project(cfg, angles, with_groups=True)
    s = cfg.spectral
    c = onz.count_scale(s.phi, s.eta, s.group_of_bin, s.n_groups, H).astype(np.float64)
    var_out = (Yg / c[None, :, None, None]).sum(axis=1)
    z = (noisy[angles] - clean[angles]) * out / np.sqrt(var_out)
    print(f"z: mean {z.mean():.4f} var {z.var():.4f} over {z.size}")
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size) + 0.01
    assert abs(z.var() - 1.0) < 0.05
    # chunking does not change a single draw
    noisy7 = fc.fcat_projections(pb, noise, angles_per_chunk=7).cpu().numpy()
    np.testing.assert_array_equal(noisy7, noisy)


def test_noisy_projections_limits(fc):
    # with the spread on: H -> infinity approaches the noiseless projections,
    # a moderate H does not
    rng = np.random.default_rng(24)
    cfg = _every_term_config(rng)
    pb = fc.upload(cfg)
    clean = fc.fcat_projections(pb, None).cpu().numpy()
    big = fc.fcat_projections(pb, fc.Noise(counts_per_pixel=1e13, seed=5)).cpu().numpy()
    got = fc.fcat_projections(pb, fc.Noise(counts_per_pixel=2.0e4, seed=5, floor=1e-6)).cpu().numpy()
    assert np.abs(big - clean).max() < 1e-4
    assert np.abs(got - clean).max() > 1e-3
    assert np.isfinite(got).all()
