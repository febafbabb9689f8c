"""FP64 oracle of the noise and projection stage.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the product library never does.

The paper adds noise through a Poisson scaling of the counts incident on the
detector (Sec. II.G), with the flood field scaled to a height of H counts per
pixel (Eq. 5: H = N_gamma / (A / A_p)) before the projections become
intensity profiles; the scatter takes Poisson noise from the counts in its
pixel; the noisy profiles go through the optical spread, are summed, and are
turned back into projections with the flood field.  Readings taken here
(the paper fixes none of these details):

* Counts of group g in a pixel have the mean lambda_g = c_g * Y_g, with Y_g
  the group signal of Eq. 3 (primary plus scatter) and
  c_g = H * Phi_g / (Phi * W_g), where Phi_g = sum_{e in g} phi_e,
  Phi = sum_e phi_e and W_g = sum_{e in g} phi_e eta_e.  An open pixel with
  I0 = 1 (Y_g = W_g) then receives H * Phi_g / Phi photons of group g and H
  in all; each photon adds eta to the signal (exact when eta is constant
  within a group, as with the paper's one energy per profile).  The scatter
  needs no draw of its own: a sum of independent Poisson variables is
  Poisson with the summed mean.
* The noisy group signal is n_g / c_g with n_g ~ Poisson(lambda_g), drawn
  before the optical spread.  A group with c_g <= 0 passes unchanged.
* The projection is -ln(max(out, floor) / flood_out), flood_out being the
  noiseless object-free flood (Y_g = W_g I0, no scatter) through the same
  spread and group sum.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written from its published
definition with Python integers.  The draw of (pixel p, group g, angle a)
uses the counters (p, g, a, j), j = 0, 1, ..., and the key (seed mod 2^32,
seed div 2^32); each counter gives two pairs (u, v) of open uniforms
(w + 1/2) / 2^32, words 0-1 first.

Poisson variates: for lambda < 16 inversion (smallest k with u <= F(k), the
CDF summed term by term); otherwise the transformed rejection method PTRS
(Hormann, "The transformed rejection method for generating Poisson random
variables", Insurance: Mathematics and Economics 12 (1993) 39-45), one
(u, v) pair per attempt.  Both in FP64.  Bounds that keep every loop finite:
at most 256 CDF terms, at most 64 attempts (then floor(lambda + 1/2)).
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = 0xFFFFFFFF
# Philox4x32 round multipliers and Weyl key increments (Salmon et al. 2011)
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
INVERSION_LIMIT = 16.0
MAX_CDF_TERMS = 256
MAX_ATTEMPTS = 64


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds: four 32-bit words from counter[4], key[2]."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in counter)
    k0, k1 = (int(x) & MASK32 for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK32,
                          (p0 >> 32) ^ c3 ^ k1, p0 & MASK32)
    return [c0, c1, c2, c3]


def uniform01(word: int) -> float:
    """(word + 1/2) / 2^32, in the open interval (0, 1)."""
    return (word + 0.5) / 4294967296.0


class UniformPairs:
    """The (u, v) pairs of one draw, in order."""

    def __init__(self, pixel: int, group: int, angle: int, seed: int):
        self.ctr = [pixel, group, angle, 0]
        self.key = [seed & MASK32, (seed >> 32) & MASK32]
        self.pending = []

    def next(self):
        if not self.pending:
            w = philox4x32_10(self.ctr, self.key)
            self.ctr[3] += 1
            self.pending = [(uniform01(w[0]), uniform01(w[1])),
                            (uniform01(w[2]), uniform01(w[3]))]
        return self.pending.pop(0)


def poisson(lam: float, pairs: UniformPairs) -> int:
    """One Poisson(lam) variate from the pairs of one draw (0 if lam <= 0 or NaN)."""
    if not lam > 0.0:
        return 0
    if lam < INVERSION_LIMIT:
        u, _ = pairs.next()
        p = math.exp(-lam)
        F = p
        k = 0
        while u > F and k < MAX_CDF_TERMS:
            k += 1
            p = p * lam / k
            F = F + p
        return k
    b = 0.931 + 2.53 * math.sqrt(lam)
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    v_r = 0.9277 - 3.6224 / (b - 2.0)
    log_lam = math.log(lam)
    for _ in range(MAX_ATTEMPTS):
        u, v = pairs.next()
        U = u - 0.5
        us = 0.5 - abs(U)
        k = math.floor((2.0 * a / us + b) * U + lam + 0.43)
        if us >= 0.07 and v <= v_r:
            return k
        if k < 0 or (us < 0.013 and v > us):
            continue
        if (math.log(v) + math.log(inv_alpha) - math.log(a / (us * us) + b)
                <= -lam + k * log_lam - math.lgamma(k + 1.0)):
            return k
    return math.floor(lam + 0.5)


def count_scale(phi, eta, group_of_bin, n_groups: int, H: float) -> np.ndarray:
    """c_g = H Phi_g / (Phi W_g) (float32 [G]); 0 where Phi_g or W_g is 0.

    Every sum runs over the bins in index order in FP64 on the float32
    inputs, so the value is fixed to the last bit before the float32 rounding.
    """
    phi = np.asarray(phi, np.float32)
    eta = np.asarray(eta, np.float32)
    grp = np.asarray(group_of_bin)
    Phi = 0.0
    for e in range(phi.size):
        Phi = Phi + float(phi[e])
    c = np.zeros(n_groups, np.float32)
    for g in range(n_groups):
        Pg = 0.0
        Wg = 0.0
        for e in range(phi.size):
            if grp[e] == g:
                Pg = Pg + float(phi[e])
                Wg = Wg + float(phi[e]) * float(eta[e])
        if Pg != 0.0 and Wg != 0.0:
            c[g] = np.float32((H * Pg) / (Phi * Wg))
    return c


def noisy_counts(Y, scale, seed: int, a0: int = 0) -> np.ndarray:
    """n[a][g][p] ~ Poisson(lambda), lambda = float32(scale[g] * Y[a][g][p]).

    Y is float32 [A][G][plane]; the draw uses the counters of (p, g, a0 + a).
    Pure Python: small inputs, or pass a few elements through ``noisy_count``.
    """
    Y = np.asarray(Y, np.float32)
    A, G, P = Y.shape
    n = np.zeros((A, G, P), np.int64)
    for a in range(A):
        for g in range(G):
            for p in range(P):
                n[a, g, p] = noisy_count(float(Y[a, g, p]), float(np.float32(scale[g])), p, g, a0 + a, seed)
    return n


def noisy_count(y: float, c: float, p: int, g: int, a: int, seed: int) -> int:
    """One element: Poisson(float32(c * y)) with the counters of (p, g, a)."""
    lam = float(np.float32(c) * np.float32(y))
    return poisson(lam, UniformPairs(p, g, a, seed))


def noisy_signal(Y, scale, seed: int, a0: int = 0) -> np.ndarray:
    """Y with noise, n / c (FP64); groups with c <= 0 unchanged."""
    Y = np.asarray(Y, np.float32)
    n = noisy_counts(Y, scale, seed, a0)
    out = Y.astype(np.float64)
    for g in range(Y.shape[1]):
        c = float(np.float32(scale[g]))
        if c > 0.0:
            out[:, g, :] = n[:, g, :] / c
    return out


def flood_groups(Wg, i0, nv: int, nu: int) -> np.ndarray:
    """Object-free, scatter-free group signals W_g I0 as [1][G][nv][nu]."""
    Wg = np.asarray(Wg, np.float64)
    I0 = np.ones((nv, nu)) if i0 is None else np.asarray(i0, np.float64).reshape(nv, nu)
    return (Wg[:, None, None] * I0[None])[None]


def projection(out, flood_out, floor: float = 0.0):
    """-ln(max(out, floor) / flood_out) per pixel (flood_out broadcast over angles)."""
    out = np.maximum(np.asarray(out, np.float64), floor)
    with np.errstate(divide="ignore"):
        return -np.log(out / np.asarray(flood_out, np.float64))
