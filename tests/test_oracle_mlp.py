"""Pins of the surrogate-network oracle.

Gradients are pinned by central finite differences of the FP64 loss; the
forward pass by a network whose output has a closed form; SiLU by its
textbook values; Adam's first step by its closed form (|step| = lr per
coordinate, up to eps); the linear term and residual targets by the
single-bin (monoenergetic) group, where the residual is exactly zero, and by
the first-order expansion for small path lengths.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def _rand_params(rng, n_in, n_out, scale=0.3):
    return rng.normal(0, scale, size=mlp.n_params(n_in, n_out))


def test_silu_values():
    z = np.array([0.0, 1.0, -1.0, 30.0, -30.0])
    np.testing.assert_allclose(mlp.silu(z), [0.0, 1 / (1 + math.exp(-1)), -1 / (1 + math.e), 30.0, 0.0],
                               atol=1e-10)
    # derivative by central differences
    zz = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.dsilu(zz), (mlp.silu(zz + h) - mlp.silu(zz - h)) / (2 * h), atol=1e-8)


def test_forward_closed_form():
    n_in, n_out = 10, 8
    W1, b1 = np.zeros((64, n_in)), np.full(64, 0.5)
    W2, b2 = np.zeros((64, 64)), np.full(64, -0.25)
    W3 = np.arange(n_out * 64, dtype=float).reshape(n_out, 64) * 1e-3
    b3 = np.linspace(-1, 1, n_out)
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = np.random.default_rng(0).uniform(0, 1, size=(5, n_in))
    out, _ = mlp.forward(p, X, n_in, n_out)
    want = W3.sum(1) * mlp.silu(-0.25) + b3
    np.testing.assert_allclose(out, np.broadcast_to(want, (5, n_out)), rtol=1e-14)


@pytest.mark.parametrize("weighted", [False, True])
def test_gradients_match_finite_differences(weighted):
    rng = np.random.default_rng(1)
    n_in, n_out, n = 10, 8, 17
    p = _rand_params(rng, n_in, n_out)
    X = rng.uniform(0, 1, size=(n, n_in))
    T = rng.normal(0, 0.2, size=(n, n_out))
    kw = {}
    if weighted:
        kw = dict(out_scale=rng.uniform(0.1, 3.0, size=n_out), weights=rng.uniform(0, 1, size=(n, n_out)))
    _, g = mlp.gradients(p, X, T, n_in, n_out, **kw)
    idx = rng.choice(p.size, size=60, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, X, T, n_in, n_out, **kw) - mlp.loss(pm, X, T, n_in, n_out, **kw)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_loss_weights():
    Y = np.array([[1.0, 1e-3], [1e-9, 2e-10], [0.5, 0.0]])      # [G][n]
    w = mlp.loss_weights(Y)
    tot = Y.sum(0)
    assert w.shape == (2, 3)                                   # [n][G]
    np.testing.assert_allclose(w[0], [1.0, min(1, 1e-9 / (1e-3 * tot[0])) ** 2, 1.0])
    np.testing.assert_allclose(w[1], [1.0, min(1, 2e-10 / (1e-3 * tot[1])) ** 2, 0.0])
    # a group at exactly the floor share weighs 1, at a tenth of it 1/100
    Y2 = np.array([[1.0, 1.0], [1e-3 / (1 - 1e-3), 1e-4 / (1 - 1e-4)]])
    np.testing.assert_allclose(mlp.loss_weights(Y2)[:, 1], [1.0, 0.01], rtol=1e-9)


def test_bf16_emulation_is_close_to_fp64():
    rng = np.random.default_rng(2)
    n_in, n_out = 10, 8
    p = _rand_params(rng, n_in, n_out)
    X = rng.uniform(0, 1, size=(64, n_in))
    o64, _ = mlp.forward(p, X, n_in, n_out)
    o16, _ = mlp.forward(p, X, n_in, n_out, bf16=True)
    # three-term split: each product is off by at most ~3 * 2^-18 of |a b|
    assert 0 < np.abs(o16 - o64).max() <= 1e-4 * np.abs(o64).max()
    # while BF16 operands alone (no lo terms) are off by ~2^-9
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    r = lambda a: mlp._b(a, True)
    h1 = mlp.silu(r(X) @ r(W1).T + b1)
    h2 = mlp.silu(r(h1) @ r(W2).T + b2)
    o_plain = r(h2) @ r(W3).T + b3
    assert np.abs(o_plain - o64).max() > 10 * np.abs(o16 - o64).max()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=20)
    g = rng.normal(size=20)
    lr = 1e-3
    p1, m, v = mlp.adam(p, g, np.zeros(20), np.zeros(20), 1, lr, eps=0.0)
    np.testing.assert_allclose(p1 - p, -lr * np.sign(g), rtol=1e-12)
    # a quadratic bowl is descended
    q = np.array([3.0])
    m = v = np.zeros(1)
    for t in range(1, 2001):
        q, m, v = mlp.adam(q, q, m, v, t, 0.05)
    assert abs(q[0]) < 0.05


def test_linear_term_and_residuals():
    rng = np.random.default_rng(4)
    M, E = 4, 6
    mu = rng.uniform(0.01, 0.1, size=(M, E))
    phi, eta = rng.uniform(0.1, 1, size=E), rng.uniform(0.2, 1, size=E)
    grp = np.array([0, 1, 1, 2, 2, 2])                  # group 0 is a single bin
    lin = mlp.linear_term(mu, phi, eta, grp, 3)
    np.testing.assert_allclose(lin[0], mu[:, 0], rtol=1e-15)
    L = rng.uniform(0, 30, size=(50, M))
    w = phi * eta
    Yp = np.stack([(w[grp == g][None, :] * np.exp(-L @ mu[:, grp == g])).sum(1) for g in range(3)])
    W = mlp.group_weights(phi, eta, grp, 3)
    r = mlp.residual_targets(L, Yp, W, lin)
    np.testing.assert_allclose(r[:, 0], 0.0, atol=1e-12)   # one bin: no beam hardening
    assert np.all(r[:, 1:] <= 1e-12)                        # Jensen: the residual is never positive
    # small path lengths: the residual is second order in L
    r_small = mlp.residual_targets(L * 1e-3, np.stack([(w[grp == g][None, :] * np.exp(-(L * 1e-3) @ mu[:, grp == g])).sum(1)
                                                       for g in range(3)]), W, lin)
    assert np.abs(r_small).max() <= 1e-5 * np.abs(r).max() + 1e-15


def test_cell_index():
    mbar = np.array([0.001, 0.02, 0.05])
    L = np.array([[100.0, 6.0, 0.0], [10.0, 0.0, 8.0], [0.0, 0.0, 0.0], [0.0, 0.0, 100.0], [50.0, 10.0, 1.0]])
    c = mlp.cell_index(L, mbar, 0.0, 2.0)
    # tau 0.22 (longest in air, but water-dominant by depth) -> bin 1; tau 0.41 -> bin 3, dominant 2; miss; tau 5 out of range;
    # tau 0.05 + 0.2 + 0.05 = 0.3 -> bin 2, dominant 1
    np.testing.assert_array_equal(c, [1 * 16 + 1, 2 * 16 + 3, -1, -1, 1 * 16 + 2])
    # the input-range test sends rays beyond the training maxima to the exact sum
    c2 = mlp.cell_index(L, mbar, 0.0, 2.0, in_scale=np.array([1 / 60.0, 1 / 20.0, 1 / 20.0]))
    np.testing.assert_array_equal(c2, [-1, 2 * 16 + 3, -1, -1, 1 * 16 + 2])


def test_mean_attenuation_and_setup_stats():
    rng = np.random.default_rng(5)
    M, E, G = 3, 12, 3
    mu = rng.uniform(0.01, 0.5, size=(M, E))
    phi, eta = rng.uniform(0.1, 1.0, E), rng.uniform(0.5, 1.0, E)
    grp = np.arange(E) * G // E
    W = mlp.group_weights(phi, eta, grp, G)
    lin = mlp.linear_term(mu, phi, eta, grp, G)
    w = phi * eta
    np.testing.assert_allclose(mlp.mean_attenuation(W, lin), (mu * w).sum(1) / w.sum(), rtol=1e-12)
    L = rng.uniform(0, 20, size=(500, M))
    L[:, 2] *= 0.5
    Y = np.stack([(w[grp == g][None, :] * np.exp(-L @ mu[:, grp == g])).sum(1) for g in range(G)])
    i_s, o_s, tmax = mlp.setup_stats(L, Y, W, lin)
    np.testing.assert_allclose(i_s, 1.0 / L.max(0), rtol=1e-12)
    assert tmax == pytest.approx((L @ ((mu * w).sum(1) / w.sum())).max(), rel=1e-12)
    r = mlp.residual_targets(L, Y, W, lin)
    wt = mlp.loss_weights(Y)
    np.testing.assert_allclose(o_s, np.sqrt((wt * r * r).sum(0) / wt.sum(0)), rtol=1e-12)


def test_setup_stats_hand_example():
    """Set-up statistics on a hand-worked three-ray example whose group
    signals have closed forms, exercising each floor and the masking.

    Two materials, five bins with phi = eta = 1 (so w_e = 1), groups
    {0, 1}, {2, 3}, {4}.  Material 0 has mu = (1, 3, 0, 1, 0.7); material 1
    never meets a ray (its max L is 0, below the 1e-6 mm floor).  For a ray
    with L = (l, 0):
      Y0 = e^-l + e^-3l,  W0 = 2, lin0 = 2    => r0 = ln 2 - l - ln(1 + e^-2l)
      Y1 = 1 + e^-l,      W1 = 2, lin1 = 1/2  => r1 = ln 2 - ln(1 + e^-l) - l/2
      Y2 = e^-0.7l,       W2 = 1, lin2 = 0.7  => r2 = 0 (one bin), so the RMS
                                                  of group 2 takes the 1e-3 floor.
    At l = 800 group 0 underflows to 0 (absorbed: weight 0, its infinite
    residual must not reach the statistics); at l = 8 group 0 carries a third
    of the 0.1% share floor, so its weight is (Y0 / (1e-3 sum Y))^2 ~ 0.112.
    The mean attenuation is (1 + 3 + 0 + 1 + 0.7) / 5 = 1.14 for material 0,
    so the top of the optical-depth range is 1.14 * 800.
    """
    mu = np.array([[1.0, 3.0, 0.0, 1.0, 0.7], [0.3, 0.3, 0.3, 0.3, 0.3]])
    phi = eta = np.ones(5)
    grp = np.array([0, 0, 1, 1, 2])
    W = mlp.group_weights(phi, eta, grp, 3)
    lin = mlp.linear_term(mu, phi, eta, grp, 3)
    l = np.array([1.0, 8.0, 800.0])
    L = np.stack([l, np.zeros(3)], axis=1)
    Y = np.stack([np.exp(-l) + np.exp(-3 * l), 1 + np.exp(-l), np.exp(-0.7 * l)])
    assert Y[0, 2] == 0.0                                    # the absorbed group
    i_s, o_s, tmax = mlp.setup_stats(L, Y, W, lin)

    assert np.all(np.isfinite(i_s)) and np.all(np.isfinite(o_s))
    np.testing.assert_allclose(i_s, [1 / 800, 1e6], rtol=1e-14)
    assert tmax == pytest.approx(1.14 * 800, rel=1e-14)
    r0 = [math.log(2) - x - math.log1p(math.exp(-2 * x)) for x in l]
    r1 = [math.log(2) - math.log1p(math.exp(-x)) - x / 2 for x in l]
    share = Y[0, 1] / (1e-3 * Y[:, 1].sum())                 # ~0.334 at l = 8
    w0 = [1.0, share ** 2, 0.0]
    assert 0.1 < w0[1] < 0.12
    rms0 = math.sqrt(sum(w * r * r for w, r in zip(w0, r0)) / sum(w0))
    rms1 = math.sqrt(sum(r * r for r in r1) / 3)
    np.testing.assert_allclose(o_s, [rms0, rms1, 1e-3], rtol=1e-12)


def test_validation_errors():
    Y = np.array([[1.0, 2.0], [1e-6, 1.0]])          # [G][n]
    P = Y.copy()
    P[1, 0] *= 2.0                                     # +100% on a group below the floor share
    P[0, 1] *= 1.0 + 1e-4
    e = mlp.validation_errors(P, Y)
    np.testing.assert_allclose(e, [1e-6 / (1e-3 * (1.0 + 1e-6)), 1e-4], rtol=1e-9)
