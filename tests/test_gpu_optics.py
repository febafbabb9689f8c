"""GPU parity of the detector-optics stage (Sec. II.B, Sec. IV.B) with the oracle.

* Effective PSF: FP64 sums, one float rounding: 1e-6 relative.
* Slit MTF: bin counts are integer work (exact); the LSF comes from the
  FP32 convolution of the slit image (1e-6 relative to its largest value);
  the MTF in FP64 from it, 2e-6 absolute.
* Richardson-Lucy: FP32 convolutions and updates, the relative error
  growing about linearly with the iterations: 2e-5 per iteration.
"""
import numpy as np
import pytest

import synth
from oracle import optics as op

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def test_effective_psf_parity(fc):
    rng = np.random.default_rng(1)
    cfg = synth.make_config(2)
    pb = fc.upload(cfg, scatter=False)
    got = fc.fcat_effective_psf(pb.spectral, pb.psf).cpu().numpy()
    s = cfg.spectral
    p64, e64 = s.phi.astype(np.float64), s.eta.astype(np.float64)
    Wg = np.array([(p64 * e64)[s.group_of_bin == g].sum() for g in range(s.n_groups)])
    ref = op.effective_psf(cfg.psf.kernels, Wg)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-9)
    del rng


@pytest.mark.parametrize("k,sig", [(15, 1.5), (7, 0.8)])
def test_slit_mtf_parity(fc, k, sig):
    p, w, tilt, over, nr, nc = 0.392, 0.3, 2.5, 10, 160, 48
    r = np.arange(k) - (k - 1) / 2
    g1 = np.exp(-0.5 * (r / sig) ** 2)
    K = np.outer(g1, g1)
    K = (K / K.sum()).astype(np.float32)
    f = np.linspace(0.0, 1.0 / p, 33)
    mtf, lsf, cnt, b_min = fc.fcat_slit_mtf(_dev(K), p, w, tilt, nr, nc, over, f)
    img = op.convolve_same(op.slit_image(nr, nc, p, w, tilt), K)
    d, ref_lsf = op.presampled_lsf(img, p, tilt, over)
    cnt = cnt.cpu().numpy()
    lsf = lsf.cpu().numpy()
    full = np.flatnonzero(cnt)
    # the same bins hold pixels, with the same counts
    h = p / over
    np.testing.assert_array_equal((b_min + full), np.round(d / h).astype(np.int64))
    np.testing.assert_allclose(lsf[full], ref_lsf, rtol=0, atol=1e-6 * ref_lsf.max())
    np.testing.assert_allclose(mtf.cpu().numpy(), op.mtf(d, ref_lsf, f), rtol=0, atol=2e-6)


@pytest.mark.parametrize("k", [7, 15])
def test_richardson_lucy_tiny_parity(fc, k):
    # k = 15 runs the ratio and the update inside the convolutions
    rng = np.random.default_rng(3)
    r = np.arange(k) - (k - 1) // 2
    K = np.exp(-0.5 * ((r[:, None] - 0.8) ** 2 / 1.2 ** 2 + (r[None, :] + 0.5) ** 2 / 0.9 ** 2))
    K = (K / K.sum()).astype(np.float32)
    d = rng.uniform(0.2, 3.0, (3, 37, 53)).astype(np.float32)
    d[1, 5:9, 10:20] = 0.0
    it = 5
    got = fc.fcat_richardson_lucy(_dev(d), _dev(K), it).cpu().numpy()
    for i in range(3):
        ref = op.richardson_lucy(d[i], K, it)
        assert np.abs(got[i] - ref).max() <= 2e-5 * it * np.abs(ref).max()
    # zero iterations return the data; flux is preserved after each step
    np.testing.assert_array_equal(fc.fcat_richardson_lucy(_dev(d), _dev(K), 0).cpu().numpy(), d)
    norm = op.convolve_same(np.ones(d.shape[1:]), K[::-1, ::-1])
    for i in range(3):
        assert abs((norm * got[i]).sum() / d[i].astype(np.float64).sum() - 1.0) < 1e-5


def test_richardson_lucy_contrast_sampled(fc):
    # the contrast workload's 360 detected profiles (64 x 1024), the effective
    # 15 x 15 PSF, 10 iterations in one call; two images against the oracle
    import torch
    cfg = synth.make_config(2)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb)
    K = fc.fcat_effective_psf(pb.spectral, pb.psf)
    it = 10
    got = fc.fcat_richardson_lucy(out, K, it)
    torch.cuda.synchronize()
    d = out[[0, 217]].cpu().numpy()
    g = got[[0, 217]].cpu().numpy()
    Kh = K.cpu().numpy()
    for i in range(2):
        ref = op.richardson_lucy(d[i], Kh, it)
        err = np.abs(g[i] - ref).max() / np.abs(ref).max()
        print(f"image {i}: max rel err {err:.2e}")
        assert err <= 2e-5 * it
