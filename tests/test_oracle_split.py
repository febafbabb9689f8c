"""Pins of the split-precision oracle (BF16 hi/lo contraction).

bf16 rounding is pinned by hand-worked values (ties to even); the split
contraction by the analytic error bound 3 * 2^-16 * sum |mu L| against the
exact FP64 product, by exactness on BF16-representable inputs, and by the
spectral sum reducing to the plain oracle when the optical depth is exact.
"""
import numpy as np

from oracle import split as sp


def test_bf16_rounding_hand_values():
    u = 2.0 ** -7                                  # BF16 spacing just above 1
    x = np.array([1.0, 1 + u, 1 + u / 2, 1 + 3 * u / 2, 1 + u / 2 + 2 ** -20, -(1 + 3 * u / 2), 3.0, 0.0],
                 dtype=np.float32)
    want = np.array([1.0, 1 + u, 1.0, 1 + 2 * u, 1 + u, -(1 + 2 * u), 3.0, 0.0], dtype=np.float32)
    np.testing.assert_array_equal(sp.bf16_rne(x), want)
    # every result has at most 8 significant bits
    r = sp.bf16_rne(np.random.default_rng(0).standard_normal(1000).astype(np.float32))
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)


def test_split_parts_reconstruct():
    x = np.random.default_rng(1).uniform(1e-3, 1e3, size=5000).astype(np.float32)
    hi, lo = sp.split(x)
    err = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -16 * np.abs(x))
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(x))


def test_split_contraction_bound_and_exact_cases():
    rng = np.random.default_rng(2)
    L = rng.uniform(0, 150, size=(400, 8)).astype(np.float32)
    mu = rng.uniform(0, 0.5, size=(8, 60)).astype(np.float32)
    exact = L.astype(np.float64) @ mu.astype(np.float64)
    Ps = sp.optical_depth_split(L, mu)
    bound = 3 * 2.0 ** -16 * (np.abs(L).astype(np.float64) @ np.abs(mu).astype(np.float64))
    assert np.all(np.abs(Ps - exact) <= bound)
    assert np.abs(Ps - exact).max() > 0          # the split form is not trivially exact
    # inputs that are already BF16 values contract exactly
    Lb, mb = sp.bf16_rne(L), sp.bf16_rne(mu)
    np.testing.assert_array_equal(sp.optical_depth_split(Lb, mb), Lb.astype(np.float64) @ mb.astype(np.float64))


def test_split_spectral_matches_plain_on_exact_inputs(orc):
    rng = np.random.default_rng(3)
    E, G, n = 24, 3, 300
    L = sp.bf16_rne(rng.uniform(0, 50, size=(n, 5)))
    mu = sp.bf16_rne(rng.uniform(0, 0.05, size=(5, E)))
    phi, eta = rng.uniform(0.1, 1, size=E), rng.uniform(0.2, 1, size=E)
    grp = np.sort(rng.integers(0, G, size=E))
    grp[:G] = np.arange(G)
    grp = np.sort(grp)
    i0, S, sb = rng.uniform(0.5, 2, size=n), rng.uniform(0, 0.2, size=n), rng.uniform(0.5, 1.5, size=E)
    Ys = sp.spectral_split(L, mu, phi, eta, grp, G, i0=i0, S=S, s_bin=sb)
    Yp = orc.spectral(L, mu, phi, eta, grp, G, i0=i0, S=S, s_bin=sb)
    np.testing.assert_allclose(Ys, Yp, rtol=1e-13)
