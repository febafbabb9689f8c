"""FP64 oracle of the learned surrogate (test infrastructure only).

The paper trains no network; it motivates simulated CBCT data for machine
learning (Sec. IV.B).  The surrogate form of the projector replaces the
primary spectral sum of Eq. 3 for one ray,

    Yprim_g = sum_{e in g} phi_e eta_e exp(-sum_m mu[m][e] L_m),

by  Yprim_g ~= W_g exp(-(sum_m lin[g][m] L_m + s_g f(x)_g)),  W_g = sum_{e in g} phi_e eta_e,

where lin[g][m] = sum_{e in g} w_e mu[m][e] / W_g is the exact first-order
(small-L) term of z_g = -ln(Yprim_g / W_g), x_m = L_m * in_scale_m, s_g a
per-group output scale, and f is the multilayer perceptron
n_in -> 64 -> 64 -> n_out with SiLU activations (silu(z) = z / (1 + e^-z)),
parameters packed as W1[64][n_in], b1[64], W2[64][64], b2[64], W3[n_out][64],
b3[n_out].  s f learns the residual r_g = z_g - sum_m lin[g][m] L_m (the
beam-hardening part of the attenuation) under a weighted squared error whose
weight min(1, Yprim_g / (1e-3 sum_g Yprim_g))^2 discounts groups that carry
less than 0.1% of the ray's signal.  The validated domain groups rays into
cells by their dominant material and mean optical depth (``cell_index``).

Everything here is plain NumPy in FP64.  ``bf16=True`` reproduces the
roundings of the GPU kernels at exactly the points where they feed the
matrix cores, so the GPU can be compared with an identical computation:
in the forward pass every product a.b of a weight and an input or hidden
activation is formed from BF16 parts, a_hi.b_hi + a_lo.b_hi + a_hi.b_lo with
v_hi = bf16(v) and v_lo = bf16(v - v_hi) (the lo.lo term is dropped); the
backward pass rounds the back-propagated signals to BF16 and uses the hi
parts of weights and activations.  The FP64 gradients are pinned by central
finite differences.  Adam follows Kingma & Ba (2015, Algorithm 1).
"""
from __future__ import annotations

import numpy as np

from .split import bf16_rne

HIDDEN = 64
CELLS = 16


def n_params(n_in: int, n_out: int) -> int:
    return HIDDEN * n_in + HIDDEN + HIDDEN * HIDDEN + HIDDEN + n_out * HIDDEN + n_out


def unpack(p, n_in: int, n_out: int):
    p = np.asarray(p, dtype=np.float64)
    o = 0

    def take(shape):
        nonlocal o
        size = int(np.prod(shape))
        a = p[o:o + size].reshape(shape)
        o += size
        return a
    W1, b1 = take((HIDDEN, n_in)), take((HIDDEN,))
    W2, b2 = take((HIDDEN, HIDDEN)), take((HIDDEN,))
    W3, b3 = take((n_out, HIDDEN)), take((n_out,))
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)])


def _b(a, on: bool):
    return bf16_rne(np.asarray(a, dtype=np.float32)).astype(np.float64) if on else np.asarray(a, np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def _hi_lo(a):
    hi = _b(a, True)
    return hi, _b(np.asarray(a, np.float64) - hi, True)


def _layer(A, W, b, bf16: bool):
    """A W^T + b; with bf16 the three-term BF16 split of every product."""
    if not bf16:
        return np.asarray(A, np.float64) @ np.asarray(W, np.float64).T + b
    Ah, Al = _hi_lo(A)
    Wh, Wl = _hi_lo(W)
    return Ah @ Wh.T + Al @ Wh.T + Ah @ Wl.T + b


def forward(p, X, n_in: int, n_out: int, bf16: bool = False):
    """Network output f(X) [n][n_out] and the cached intermediates (inputs
    and activations as the backward pass uses them: BF16 hi parts when bf16)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    X = np.asarray(X, np.float64)
    Z1 = _layer(X, W1, b1, bf16)
    H1 = silu(Z1)
    Z2 = _layer(H1, W2, b2, bf16)
    H2 = silu(Z2)
    out = _layer(H2, W3, b3, bf16)
    return out, (_b(X, bf16), Z1, _b(H1, bf16), Z2, _b(H2, bf16))


def _scales(out_scale, weights, shape):
    s = np.ones(shape[1]) if out_scale is None else np.asarray(out_scale, np.float64)
    w = np.ones(shape) if weights is None else np.asarray(weights, np.float64)
    return s, w


def loss(p, X, T, n_in: int, n_out: int, bf16: bool = False, out_scale=None, weights=None) -> float:
    """Weighted mean squared error  mean(w (s f - T)^2)  over all samples and outputs."""
    out, _ = forward(p, X, n_in, n_out, bf16)
    s, w = _scales(out_scale, weights, out.shape)
    return float(np.mean(w * (s * out - np.asarray(T, np.float64)) ** 2))


def gradients(p, X, T, n_in: int, n_out: int, bf16: bool = False, out_scale=None, weights=None):
    """(loss, dloss/dp) by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    out, (Xb, Z1, H1, Z2, H2) = forward(p, X, n_in, n_out, bf16)
    T = np.asarray(T, np.float64)
    n = out.shape[0]
    s, w = _scales(out_scale, weights, out.shape)
    d = s * out - T
    dO = 2.0 * w * d * s / (n * n_out)
    dOb = _b(dO, bf16)
    gW3 = dOb.T @ H2
    gb3 = dO.sum(0)
    dH2 = dOb @ _b(W3, bf16)
    dZ2 = dH2 * dsilu(Z2)
    dZ2b = _b(dZ2, bf16)
    gW2 = dZ2b.T @ H1
    gb2 = dZ2.sum(0)
    dH1 = dZ2b @ _b(W2, bf16)
    dZ1 = dH1 * dsilu(Z1)
    dZ1b = _b(dZ1, bf16)
    gW1 = dZ1b.T @ Xb
    gb1 = dZ1.sum(0)
    return float(np.mean(w * d ** 2)), pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------- surrogate pieces

def group_weights(phi, eta, group_of_bin, n_groups: int) -> np.ndarray:
    w = np.asarray(phi, np.float64) * np.asarray(eta, np.float64)
    return np.array([w[np.asarray(group_of_bin) == g].sum() for g in range(n_groups)])


def linear_term(mu, phi, eta, group_of_bin, n_groups: int) -> np.ndarray:
    """lin[g][m] = sum_{e in g} w_e mu[m][e] / W_g."""
    w = np.asarray(phi, np.float64) * np.asarray(eta, np.float64)
    mu = np.asarray(mu, np.float64)
    grp = np.asarray(group_of_bin)
    out = np.zeros((n_groups, mu.shape[0]))
    for g in range(n_groups):
        sel = grp == g
        out[g] = (mu[:, sel] * w[sel]).sum(1) / w[sel].sum()
    return out


def residual_targets(L, Yprim, W, lin) -> np.ndarray:
    """r[n][G] = -ln(Yprim / W) - L lin^T."""
    L = np.asarray(L, np.float64)
    z = -np.log(np.asarray(Yprim, np.float64).T / np.asarray(W, np.float64)[None, :])
    return z - L @ np.asarray(lin, np.float64).T


SHARE_FLOOR = 1e-3


def loss_weights(Yprim) -> np.ndarray:
    """w[n][G] = min(1, Yprim_g / (1e-3 sum_g Yprim_g))^2 for Yprim [G][n]."""
    Y = np.asarray(Yprim, np.float64).T
    return np.minimum(1.0, Y / (SHARE_FLOOR * Y.sum(1, keepdims=True))) ** 2


def predict_yprim(p, L, in_scale, lin, W, n_out: int, bf16: bool = False, out_scale=None) -> np.ndarray:
    """Yprim[G][n] predicted by the surrogate."""
    L = np.asarray(L, np.float64)
    X = L * np.asarray(in_scale, np.float64)[None, :]
    r, _ = forward(p, X, L.shape[1], n_out, bf16)
    if out_scale is not None:
        r = r * np.asarray(out_scale, np.float64)[None, :]
    z = L @ np.asarray(lin, np.float64).T + r
    return (np.asarray(W, np.float64)[None, :] * np.exp(-z)).T


def mean_attenuation(W, lin) -> np.ndarray:
    """mbar[m] = sum_g W_g lin[g][m] / sum_g W_g = sum_e w_e mu[m][e] / sum_e w_e."""
    W = np.asarray(W, np.float64)
    return W @ np.asarray(lin, np.float64) / W.sum()


def cell_index(L, mbar, cell_lo: float, cell_hi: float, in_scale=None) -> np.ndarray:
    """Validation cell of each ray: argmax_m mbar_m L_m * 16 + bin of the mean
    optical depth tau = sum_m mbar_m L_m over [cell_lo, cell_hi); -1 for a miss,
    a depth outside the bins, or (with in_scale) some L_m in_scale_m > 1.

    The cell is an integer decision taken from floating point, so it is taken
    here in the kernels' precision: FP32 products and sums in material order,
    FP32 bin arithmetic.
    """
    f = np.float32
    L = np.asarray(L, f)
    t = L * np.asarray(mbar, f)[None, :]
    tau = np.zeros(L.shape[0], f)
    for m in range(L.shape[1]):
        tau = tau + t[:, m]
    dom = np.argmax(t, axis=1)
    b = np.floor((f(CELLS) * (tau - f(cell_lo))) / (f(cell_hi) - f(cell_lo)))
    ok = (L.sum(1, dtype=np.float64) > 0) & (b >= 0) & (b < CELLS)
    if in_scale is not None:
        ok &= np.all(L * np.asarray(in_scale, f)[None, :] <= f(1.0), axis=1)
    return np.where(ok, dom * CELLS + np.clip(b, 0, CELLS - 1).astype(np.int64), -1)


def validation_errors(pred, Yprim) -> np.ndarray:
    """Per ray max_g |pred_g - Y_g| / max(Y_g, 1e-3 sum_g Y_g), for [G][n] arrays."""
    P = np.asarray(pred, np.float64)
    Y = np.asarray(Yprim, np.float64)
    floor = SHARE_FLOOR * Y.sum(0, keepdims=True)
    return (np.abs(P - Y) / np.maximum(Y, floor)).max(0)


def setup_stats(L, Yprim, W, lin):
    """(in_scale, out_scale, tau_max) of a training set: 1 / max L_m (floor
    1e-6 mm), the weighted RMS of the residual targets (floor 1e-3) and the
    largest mean optical depth."""
    L = np.asarray(L, np.float64)
    in_scale = 1.0 / np.maximum(L.max(0), 1e-6)
    w = loss_weights(Yprim)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = residual_targets(L, Yprim, W, lin)
    r = np.where(w > 0, r, 0.0)
    out_scale = np.maximum(1e-3, np.sqrt((w * r * r).sum(0) / np.maximum(w.sum(0), 1e-30)))
    tau_max = float((L @ mean_attenuation(W, lin)).max())
    return in_scale, out_scale, tau_max
