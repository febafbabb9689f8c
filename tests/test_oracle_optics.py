"""Pins of the detector-optics oracle (oracle/optics.py): effective PSF,
tilted-slit presampled MTF (Sec. II.B) and Richardson-Lucy deconvolution
(Sec. IV.B; Richardson 1972, Lucy 1974).

Expected values: brute-force supersampling of the slit's pixel coverage;
the strip's area per row; the MTF of an unblurred slit (product of the
slit's and the pixel aperture's sinc functions) and of a Gaussian PSF (a
Gaussian factor more); the RL fixed point on noiseless data, its flux
preservation and its non-decreasing Poisson likelihood.
"""
import math

import numpy as np
import pytest
import scipy.signal

from oracle import optics as op


def _sinc(x):
    return np.sinc(x)            # sin(pi x) / (pi x)


def test_effective_psf_weights():
    rng = np.random.default_rng(1)
    K = rng.random((3, 5, 5))
    K /= K.sum(axis=(1, 2), keepdims=True)
    W = np.array([0.4, 1.0, 0.6])          # normalised by their sum, 2
    E = op.effective_psf(K, W)
    np.testing.assert_allclose(E, 0.2 * K[0] + 0.5 * K[1] + 0.3 * K[2], rtol=1e-14)
    assert abs(E.sum() - 1.0) < 1e-14


def test_convolve_same_is_scipy():
    rng = np.random.default_rng(2)
    img, K = rng.random((23, 31)), rng.random((7, 7))
    np.testing.assert_allclose(op.convolve_same(img, K), scipy.signal.convolve2d(img, K, mode="same"), rtol=1e-12)


def test_slit_coverage_exact():
    p, w, tilt = 0.4, 0.3, 2.5
    img = op.slit_image(40, 24, p, w, tilt)
    assert img.min() >= -1e-12 and img.max() <= 1.0 + 1e-12
    # each row band of height p holds the strip's area (w / cos t) p
    np.testing.assert_allclose(img.sum(axis=1) * p * p, w / math.cos(math.radians(tilt)) * p, rtol=1e-12)
    # brute force: 400 x 400 sub-samples of a few pixels
    t = math.radians(tilt)
    n = np.array([math.cos(t), math.sin(t)])
    for (i, j) in [(20, 11), (20, 12), (5, 12), (33, 13), (0, 0)]:
        cx, cy = (j - 11.5) * p, (i - 19.5) * p
        s = (np.arange(400) + 0.5) / 400 * p - p / 2
        X, Y = np.meshgrid(cx + s, cy + s)
        frac = (np.abs(n[0] * X + n[1] * Y) <= w / 2).mean()
        assert abs(img[i, j] - frac) < 4e-3, (i, j, img[i, j], frac)


def test_unblurred_slit_mtf_is_the_aperture():
    # no spread: the presampled LSF is the strip seen through the pixel, whose
    # transfer is sinc(w f) sinc(p cos t f) sinc(p sin t f); binning adds sinc(h f)
    p, w, tilt, over = 0.4, 0.3, 2.5, 10
    img = op.slit_image(256, 64, p, w, tilt)
    d, lsf = op.presampled_lsf(img, p, tilt, over)
    t = math.radians(tilt)
    h = p / over
    assert abs(lsf.sum() * h - w) < 0.01 * w
    # the slit is centred on d = 0, and so is its LSF (bins centred on multiples of h)
    assert abs((d * lsf).sum() / lsf.sum()) < 0.05 * h
    f = np.linspace(0.0, 1.0 / p, 21)
    want = np.abs(_sinc(w * f) * _sinc(p * math.cos(t) * f) * _sinc(p * math.sin(t) * f) * _sinc(h * f))
    got = op.mtf(d, lsf, f)
    np.testing.assert_allclose(got, want, atol=0.01)


def test_gaussian_psf_mtf():
    p, w, tilt, over, sig = 0.4, 0.3, 2.5, 10, 1.5      # sigma in pixels
    k = 15
    r = np.arange(k) - (k - 1) / 2
    g1 = np.exp(-0.5 * (r / sig) ** 2)
    K = np.outer(g1, g1)
    K /= K.sum()
    img = op.convolve_same(op.slit_image(256, 64, p, w, tilt), K)
    d, lsf = op.presampled_lsf(img[16:-16], p, tilt, over)
    t = math.radians(tilt)
    f = np.linspace(0.0, 1.0 / p, 21)
    aperture = np.abs(_sinc(w * f) * _sinc(p * math.cos(t) * f) * _sinc(p * math.sin(t) * f) * _sinc(p / over * f))
    # the kernel is the Gaussian sampled on the pixel grid: its transfer is the
    # Gaussian's periodised with period 1 / p
    gauss = sum(np.exp(-2 * math.pi ** 2 * (sig * p) ** 2 * (f - m / p) ** 2) for m in (-1, 0, 1))
    want = aperture * gauss
    np.testing.assert_allclose(op.mtf(d, lsf, f), want, atol=0.01)


def _loglik(d, c):
    return float((d * np.log(np.maximum(c, 1e-300)) - c).sum())


def test_richardson_lucy_fixed_point_flux_and_likelihood():
    rng = np.random.default_rng(5)
    k = 7
    r = np.arange(k) - 3
    # an asymmetric kernel, so that convolution and correlation differ
    K = np.exp(-0.5 * ((r[:, None] - 0.8) ** 2 / 1.2 ** 2 + (r[None, :] + 0.5) ** 2 / 0.9 ** 2))
    K /= K.sum()
    u_true = rng.uniform(0.5, 2.0, (20, 26))
    d = op.convolve_same(u_true, K)
    # the true image is a fixed point on noiseless data
    np.testing.assert_allclose(op.richardson_lucy(d, K, 1, u0=u_true), u_true, rtol=1e-12)
    # flux: sum of (K^T 1) u after a step equals sum d; the likelihood never falls
    norm = op.convolve_same(np.ones_like(d), K[::-1, ::-1])
    u = d.copy()
    ll = _loglik(d, op.convolve_same(u, K))
    for _ in range(6):
        u = op.richardson_lucy(d, K, 1, u0=u)
        assert abs((norm * u).sum() / d.sum() - 1.0) < 1e-12
        ll2 = _loglik(d, op.convolve_same(u, K))
        assert ll2 >= ll - 1e-9
        ll = ll2
    # and the iterates move towards the truth
    assert np.abs(u - u_true).mean() < np.abs(d - u_true).mean()
