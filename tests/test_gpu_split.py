"""GPU parity of the split-precision form (L . mu on matrix cores, BF16 hi/lo).

Two bars: against the split oracle (same BF16 parts, FP64 sums) the kernel
may differ only by FP32 accumulation and the fast exp (5e-6 relative);
against the exact FP64 oracle the form must stay within 1e-3 relative.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import rel_err
from oracle import split as osplit

pytestmark = pytest.mark.gpu


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("cfg_n,n_mat", [(1, None), (2, None), (3, None), (2, 12), (2, 27)])
def test_split_spectral(fc, cfg_n, n_mat):
    import torch
    cfg = synth.make_config(cfg_n)
    s = cfg.spectral
    rng = np.random.default_rng(7 + cfg_n)
    mu = s.mu
    if n_mat is not None:                      # more materials: 2 or 3 k blocks on the matrix cores
        mu = np.concatenate([s.mu] * (n_mat // s.n_mat + 1))[:n_mat] * rng.uniform(0.8, 1.2, size=(n_mat, 1))
        mu = mu.astype(np.float32)
    M = mu.shape[0]
    n = 4096 + 29
    L = (rng.uniform(0, 1, size=(n, M)) ** 3 * 60.0 / M * 8).astype(np.float32)
    L[:40] = 0.0
    i0 = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    S = rng.uniform(0.0, 0.2, size=n).astype(np.float32)
    sp = fc.Spectral(_t(torch, mu), _t(torch, s.phi), _t(torch, s.eta), s.n_groups, s.group_of_bin)
    Y = fc.fcat_spectral(_t(torch, L), sp, i0=_t(torch, i0), S=_t(torch, S), mode="split_bf16").cpu().numpy()
    ref_split = osplit.spectral_split(L, mu, s.phi, s.eta, s.group_of_bin, s.n_groups, i0=i0, S=S)
    ref = oracle.spectral(L, mu, s.phi, s.eta, s.group_of_bin, s.n_groups, i0=i0, S=S)
    e_split, e_exact = rel_err(Y, ref_split).max(), rel_err(Y, ref).max()
    print(f"config {cfg_n} M={M}: vs split oracle {e_split:.2e}, vs exact {e_exact:.2e}")
    assert e_split <= 5e-6
    assert e_exact <= 1e-3


def test_split_project_tiny_and_contrast(fc):
    for n, angles in ((1, list(range(45))), (2, [0, 91, 359])):
        cfg = synth.make_config(n)
        pb = fc.upload(cfg)
        out = fc.fcat_project(pb, mode="split_bf16").cpu().numpy()
        plain = fc.fcat_project(pb).cpu().numpy()
        ref = oracle.project(cfg, angles)
        err = rel_err(out[angles], ref)
        print(f"config {n}: split vs oracle max {err.max():.2e} rms {np.sqrt((err ** 2).mean()):.2e}; "
              f"split vs plain {rel_err(out, plain).max():.2e}")
        assert err.max() <= 1e-3
        assert rel_err(out, plain).max() <= 1e-3


def test_split_project_head_sampled(fc):
    import torch
    cfg = synth.make_config(3)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb, mode="split_bf16")
    sample = [5, 400]
    o = out[sample].cpu().numpy()
    del out, pb
    torch.cuda.empty_cache()
    err = rel_err(o, oracle.project(cfg, sample))
    print(f"head split: max {err.max():.2e}")
    assert err.max() <= 1e-3


@pytest.mark.parametrize("k,nu", [(3, 101), (15, 101), (17, 101), (19, 101), (1, 100), (15, 100), (17, 100)])
def test_split_psf_ragged_detector(fc, k, nu):
    """The split form's optical spread runs on the matrix cores for k <= 17 (banded
    Toeplitz operands, BF16 hi/lo); k = 19 takes the FP32 kernel.  Ragged detector
    (nu x 21 pixels: partial 64 x 64 tiles in both directions), 4 groups; nu = 100
    takes the 16-byte tile loads, nu = 101 the 4-byte ones."""
    rng = np.random.default_rng(100 + k)
    cfg = synth.make_config(1)
    cfg.geometry.nu, cfg.geometry.nv = nu, 21
    cfg.spectral.n_groups = 4
    cfg.spectral.group_of_bin = synth.contiguous_groups(cfg.spectral.n_energy, 4)
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 4, k))
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb, mode="split_bf16").cpu().numpy()
    plain = fc.fcat_project(pb).cpu().numpy()
    angles = list(range(0, 45, 4))
    ref = oracle.project(cfg, angles)
    e_or, e_pl = rel_err(out[angles], ref).max(), rel_err(out, plain).max()
    print(f"k={k}: split vs oracle {e_or:.2e}, split vs plain {e_pl:.2e}")
    assert e_or <= 1e-3 and e_pl <= 1e-4
