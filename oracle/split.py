"""FP64 oracle of the split-precision contraction (test infrastructure only).

The split-precision form evaluates the per-energy optical depth
P_e = sum_m mu[m][e] L_m (Sec. II.F: one projection per energy of a labelled
phantom) from BF16 parts:

    x_hi = bf16(x)            (round to nearest, ties to even)
    x_lo = bf16(x - x_hi)     (x - x_hi is exact in FP32)
    P_e ~= sum_m mu_hi L_hi + mu_lo L_hi + mu_hi L_lo

This module writes that definition out in FP64 on the rounded parts, so a
GPU kernel that multiplies the same BF16 values exactly and accumulates in
FP32 must agree with it to FP32 accumulation error; against the exact
optical depth it differs by at most 3 * 2^-16 * sum_m |mu_m L_m| (the dropped
lo * lo term and the rounding of the two residuals).  The spectral weighting
then follows Eq. 3 exactly as in the plain oracle.
"""
from __future__ import annotations

import numpy as np

BF16_UNIT = 2.0 ** -8          # unit roundoff of BF16 (8 significant bits)


def bf16_rne(x) -> np.ndarray:
    """Round float32 values to BF16 (nearest, ties to even), returned as float32."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).reshape(x.shape)


def split(x):
    """(hi, lo) BF16 parts of float32 x, both as float32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne(x - hi)          # exact difference in float32
    return hi, lo


def optical_depth_split(L, mu) -> np.ndarray:
    """P[r][e] from the BF16 parts of L[r][m] and mu[m][e], summed in FP64."""
    Lh, Ll = (a.astype(np.float64) for a in split(L))
    mh, ml = (a.astype(np.float64) for a in split(mu))
    return Lh @ mh + Lh @ ml + Ll @ mh


def spectral_split(L, mu, phi, eta, group_of_bin, n_groups: int, i0=None, S=None, s_bin=None) -> np.ndarray:
    """Y[G][n] of Eq. 3 with the split-precision optical depth."""
    L = np.asarray(L, dtype=np.float32).reshape(-1, np.shape(mu)[0])
    P = optical_depth_split(L, np.asarray(mu, dtype=np.float32))
    w = np.asarray(phi, dtype=np.float64) * np.asarray(eta, dtype=np.float64)
    n = L.shape[0]
    flood = np.ones(n) if i0 is None else np.asarray(i0, dtype=np.float64).reshape(-1)
    sc = np.zeros(n) if S is None else np.asarray(S, dtype=np.float64).reshape(-1)
    sb = np.ones(len(w)) if s_bin is None else np.asarray(s_bin, dtype=np.float64)
    grp = np.asarray(group_of_bin)
    Y = np.zeros((n_groups, n))
    T = np.exp(-P)
    for e in range(len(w)):
        Y[grp[e]] += w[e] * (flood * T[:, e] + sb[e] * sc)
    return Y
