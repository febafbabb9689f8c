"""GPU parity of the spectral sum (Eq. 3) and the optical spread (Sec. II.G)
with the FP64 oracle, called through the C ABI on seeded inputs."""
import numpy as np
import pytest

import oracle
import synth
from conftest import rel_err

pytestmark = pytest.mark.gpu


def _spectral(fc, s, torch, gob=None):
    return fc.Spectral(torch.as_tensor(s.mu, device="cuda"), torch.as_tensor(s.phi, device="cuda"),
                       torch.as_tensor(s.eta, device="cuda"), s.n_groups,
                       s.group_of_bin if gob is None else gob)


@pytest.mark.parametrize("cfg_n", [1, 2, 3])
def test_spectral_matches_oracle(fc, cfg_n):
    import torch
    cfg = synth.make_config(cfg_n)
    s = cfg.spectral
    rng = np.random.default_rng(cfg_n)
    n = 4096 + 37                                     # several blocks and a ragged tail
    chord = 2.0 * np.abs(cfg.phantom.labels.shape[-1] * cfg.phantom.dx) / 2
    L = (rng.uniform(0, 1, size=(n, s.n_mat)) ** 3 * chord / 2).astype(np.float32)
    L[:50] = 0.0                                      # misses
    i0 = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    S = rng.uniform(0.0, 0.2, size=n).astype(np.float32)
    sb = rng.uniform(0.5, 1.5, size=s.n_energy).astype(np.float32)
    sp = _spectral(fc, s, torch)
    t = lambda a: torch.as_tensor(a, device="cuda")
    Y = fc.fcat_spectral(t(L), sp, i0=t(i0), S=t(S), s_bin=t(sb)).cpu().numpy()
    ref = oracle.spectral(L, s.mu, s.phi, s.eta, s.group_of_bin, s.n_groups, i0=i0, S=S, s_bin=sb)
    err = rel_err(Y, ref)
    print(f"config {cfg_n}: spectral max rel err {err.max():.3e}")
    assert err.max() <= 1e-5
    # no flood, no scatter
    Y2 = fc.fcat_spectral(t(L), sp).cpu().numpy()
    ref2 = oracle.spectral(L, s.mu, s.phi, s.eta, s.group_of_bin, s.n_groups)
    assert rel_err(Y2, ref2).max() <= 1e-5


@pytest.mark.parametrize("n_mat", [3, 12, 27])
def test_spectral_material_counts_and_group_maps(fc, n_mat):
    import torch
    rng = np.random.default_rng(n_mat)
    E, G, n = 77, 5, 999
    mu = rng.uniform(0, 0.05, size=(n_mat, E)).astype(np.float32)
    phi = rng.uniform(0, 1, size=E).astype(np.float32)
    eta = rng.uniform(0.1, 1, size=E).astype(np.float32)
    gob = np.sort(np.concatenate([np.arange(G), rng.integers(0, G, size=E - G)])).astype(np.int32)
    L = rng.uniform(0, 30, size=(n, n_mat)).astype(np.float32)
    t = lambda a: torch.as_tensor(a, device="cuda")
    sp = fc.Spectral(t(mu), t(phi), t(eta), G, gob)
    Y = fc.fcat_spectral(t(L), sp).cpu().numpy()
    ref = oracle.spectral(L, mu, phi, eta, gob, G)
    assert rel_err(Y, ref).max() <= 1e-5
    # default contiguous map
    sp0 = fc.Spectral(t(mu), t(phi), t(eta), G, None)
    Y0 = fc.fcat_spectral(t(L), sp0).cpu().numpy()
    ref0 = oracle.spectral(L, mu, phi, eta, synth.contiguous_groups(E, G), G)
    assert rel_err(Y0, ref0).max() <= 1e-5


@pytest.mark.parametrize("k", [15, 1, 5, 31])
def test_psf_matches_oracle(fc, k):
    import torch
    rng = np.random.default_rng(k)
    A, G, nv, nu = 3, 8, 37, 101                      # ragged in both detector directions
    Y = rng.uniform(0, 1, size=(A, G, nv, nu)).astype(np.float32)
    K = synth.gaussian_psfs(rng, G, k) if k > 1 else rng.uniform(0.5, 1, size=(G, 1, 1)).astype(np.float32)
    out = fc.fcat_psf(torch.as_tensor(Y, device="cuda"), fc.Psf(torch.as_tensor(K, device="cuda")))
    ref = oracle.psf(Y, K)
    err = rel_err(out.cpu().numpy(), ref)
    print(f"k={k}: psf max rel err {err.max():.3e}")
    assert err.max() <= 1e-5


def test_psf_asymmetric_kernel_and_delta(fc):
    import torch
    rng = np.random.default_rng(3)
    A, G, nv, nu, k = 2, 3, 70, 130, 15
    Y = rng.uniform(0, 1, size=(A, G, nv, nu)).astype(np.float32)
    K = np.zeros((G, k, k), np.float32)
    K[0, 7, 7] = 1.0                                  # identity
    K[1, 2, 11] = 1.0                                 # pure shift: pins the flip
    K[2] = rng.uniform(0, 1, size=(k, k))
    t = lambda a: torch.as_tensor(a, device="cuda")
    out = fc.fcat_psf(t(Y), fc.Psf(t(K))).cpu().numpy()
    ref = oracle.psf(Y, K)
    assert rel_err(out, ref).max() <= 1e-5
    K1 = np.zeros((1, k, k), np.float32)
    K1[0, 7, 7] = 1.0
    ident = fc.fcat_psf(t(Y[:, :1].copy()), fc.Psf(t(K1))).cpu().numpy()
    np.testing.assert_array_equal(ident, Y[:, 0])


def test_exp_accuracy_over_the_optical_depth_range(fc):
    """One material, one bin, mu = phi = eta = 1: the spectral sum returns
    exp(-P) for P = L, so this pins the device exponential against FP64 over
    the optical depths FP32 can hold as normal numbers (P in [0, 87]), then
    over the results below the smallest normal number (which may be flushed
    to 0), negative depths, large finite depths and NaN.  Infinite depths,
    depths beyond 2e38 and negative ones below -88 come only from non-finite
    or negative inputs and are not defined.

    Bound: the sum forms its exponent in base 2, x = fl(mu log2 e) L, two
    roundings of relative 2^-24 each, so x is off by at most 2^-23 x, which
    moves 2^-x by a relative ln 2 * 2^-23 x = 2^-23 P; the hardware 2^-x adds
    about one ulp (2.5e-7 allowed).  An FP32 optical depth is itself only
    known to half an ulp, a relative 2^-24 P in exp(-P), so the bound is
    twice what the input's own rounding gives."""
    import torch
    P = np.linspace(0.0, 87.0, 400001).astype(np.float32)
    L = torch.as_tensor(P[:, None].copy()).cuda()
    one = lambda *shape: torch.ones(*shape, dtype=torch.float32, device="cuda")
    sp = fc.Spectral(mu=one(1, 1), phi=one(1), eta=one(1), n_groups=1)
    Y = fc.fcat_spectral(L, sp).cpu().numpy()[0].astype(np.float64)
    ref = np.exp(-P.astype(np.float64))
    rel = np.abs(Y - ref) / ref
    bound = 2.5e-7 + P.astype(np.float64) * 2.0 ** -23
    print(f"exp(-P), P in [0, 87]: max rel err {rel.max():.2e}, max share of the bound {(rel / bound).max():.3f}")
    assert (rel <= bound).all()
    # below the normal range, negative depths, large finite depths, NaN
    P = np.concatenate([np.linspace(87.0, 105.0, 20001), np.linspace(-88.5, 0.0, 2001),
                        [110.0, 1e3, 1e5, 1e6, 1e7, 1e30, np.nan]]).astype(np.float32)
    L = torch.as_tensor(P[:, None].copy()).cuda()
    Y = fc.fcat_spectral(L, sp).cpu().numpy()[0]
    with np.errstate(over="ignore"):
        ref = np.exp(-P.astype(np.float64))
    fin = np.isfinite(P)
    err = np.abs(Y[fin].astype(np.float64) - ref[fin])
    bound = (2.5e-7 + np.abs(P[fin].astype(np.float64)) * 2.0 ** -23) * ref[fin]
    assert np.all(err <= np.maximum(bound, 2.0 ** -126))
    assert np.all(Y[-7:-1] == 0.0) and np.isnan(Y[-1])
