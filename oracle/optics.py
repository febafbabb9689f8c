"""FP64 oracle of the detector MTF and of Richardson-Lucy deconvolution.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the product library never does.

Sec. II.B: the energy-dependent optical spread functions, weighted by the
detector's energy deposition efficiency times the incident spectrum, give a
hypothetical PSF; convolved with an idealised 0.3 mm slit tilted by 2.5
degrees it gives a line spread function, presampled to estimate the MTF.
Sec. IV.B: with the PSF known, Richardson-Lucy deconvolution (Richardson
1972; Lucy 1974) of the projection images sharpens the reconstruction.
Readings taken here:

* effective PSF: K = sum_g W_g K_g / sum_g W_g over the energy groups
  (W_g = sum_{e in g} phi_e eta_e);
* slit image: each detector pixel (pitch p, centre of pixel (i, j) at
  ((j - (nc - 1)/2) p, (i - (nr - 1)/2) p), j the column) holds the exact
  fraction of its area inside the strip |(x, y) . n| <= w / 2 with
  n = (cos t, sin t), t the tilt from the detector columns; then the image
  is convolved with K (zero outside, as for the projector);
* presampled LSF: every pixel of the blurred slit image is binned by the
  signed distance d = (x, y) . n of its centre to the slit's centre line,
  in bins of p / oversample centred on multiples of it; the LSF is the mean
  per bin (empty bins are left out);
* MTF(f) = |sum_b LSF_b exp(-2 pi i f d_b)| / |sum_b LSF_b| over the bins,
  with no slit-width or pixel-aperture correction;
* Richardson-Lucy on an image d >= 0 with kernel K (convolution with zeros
  outside): u <- u * (K^T * (d / (K * u))) / (K^T * 1), K^T the flipped
  kernel (correlation), the ratio taken as 0 where K * u = 0, starting from
  u = d.  The division by K^T * 1 keeps the update flux-preserving at the
  image border, where part of K falls outside.
"""
from __future__ import annotations

import math

import numpy as np


def effective_psf(kernels, Wg) -> np.ndarray:
    """sum_g W_g K_g / sum_g W_g."""
    K = np.asarray(kernels, np.float64)
    W = np.asarray(Wg, np.float64)
    return (W[:, None, None] * K).sum(axis=0) / W.sum()


def convolve_same(img, K) -> np.ndarray:
    """(K * img)[i][j] = sum_{p,q} K[p][q] img[i - p + c][j - q + c], zero outside, c = (k - 1)/2."""
    img = np.asarray(img, np.float64)
    K = np.asarray(K, np.float64)
    k = K.shape[0]
    c = (k - 1) // 2
    nr, nc = img.shape
    pad = np.zeros((nr + 2 * c, nc + 2 * c))
    pad[c:c + nr, c:c + nc] = img
    out = np.zeros((nr, nc))
    for p in range(k):
        for q in range(k):
            # img[i - p + c][j - q + c] = pad[i - p + 2c][j - q + 2c]
            out += K[p, q] * pad[2 * c - p:2 * c - p + nr, 2 * c - q:2 * c - q + nc]
    return out


def _halfplane_area(t, a, b, p):
    """Area of the p x p square [-p/2, p/2]^2 where a x + b y <= t (a, b != 0)."""
    # a x + b y over the square is the sum of two uniform variables of widths
    # |a| p and |b| p: its distribution function is a difference of ramps squared
    A, B = abs(a) * p, abs(b) * p
    s0 = -(A + B) / 2.0
    r = lambda u: np.maximum(u, 0.0) ** 2
    return (r(t - s0) - r(t - s0 - A) - r(t - s0 - B) + r(t - s0 - A - B)) / (2.0 * A * B) * p * p


def slit_image(n_rows: int, n_cols: int, pitch: float, width: float, tilt_deg: float) -> np.ndarray:
    """Fraction of each pixel's area inside the tilted strip (tilt in (0, 90) degrees)."""
    t = math.radians(tilt_deg)
    nx, ny = math.cos(t), math.sin(t)
    x = (np.arange(n_cols) - (n_cols - 1) / 2.0) * pitch
    y = (np.arange(n_rows) - (n_rows - 1) / 2.0) * pitch
    d = nx * x[None, :] + ny * y[:, None]          # distance of each pixel centre
    hi = _halfplane_area(width / 2.0 - d, nx, ny, pitch)
    lo = _halfplane_area(-width / 2.0 - d, nx, ny, pitch)
    return (hi - lo) / (pitch * pitch)


def presampled_lsf(image, pitch: float, tilt_deg: float, oversample: int):
    """(d_b, LSF_b) of the non-empty bins, d_b = b pitch / oversample."""
    img = np.asarray(image, np.float64)
    n_rows, n_cols = img.shape
    t = math.radians(tilt_deg)
    x = (np.arange(n_cols) - (n_cols - 1) / 2.0) * pitch
    y = (np.arange(n_rows) - (n_rows - 1) / 2.0) * pitch
    d = math.cos(t) * x[None, :] + math.sin(t) * y[:, None]
    h = pitch / oversample
    b = np.floor(d / h + 0.5).astype(np.int64)
    bins = np.unique(b)
    lsf = np.array([img[b == k].mean() for k in bins])
    return bins * h, lsf


def mtf(d, lsf, freqs) -> np.ndarray:
    """|sum_b LSF_b e^{-2 pi i f d_b}| / |sum_b LSF_b|."""
    d = np.asarray(d, np.float64)
    lsf = np.asarray(lsf, np.float64)
    f = np.asarray(freqs, np.float64)
    ph = -2.0 * math.pi * f[:, None] * d[None, :]
    re = (lsf[None, :] * np.cos(ph)).sum(axis=1)
    im = (lsf[None, :] * np.sin(ph)).sum(axis=1)
    return np.hypot(re, im) / abs(lsf.sum())


def richardson_lucy(d, K, iterations: int, u0=None) -> np.ndarray:
    """Richardson-Lucy iterations on one image (see the module notes)."""
    d = np.asarray(d, np.float64)
    K = np.asarray(K, np.float64)
    Kt = K[::-1, ::-1]
    norm = convolve_same(np.ones_like(d), Kt)
    u = d.copy() if u0 is None else np.asarray(u0, np.float64).copy()
    for _ in range(iterations):
        c = convolve_same(u, K)
        ratio = np.where(c > 0.0, d / np.where(c > 0.0, c, 1.0), 0.0)
        u = u * convolve_same(ratio, Kt) / norm
    return u
