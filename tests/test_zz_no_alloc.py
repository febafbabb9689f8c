"""fcat_spectral_static (no workspace: its tables in the library's static
device scratch) against fcat_spectral with a caller workspace, through the C
ABI.  Both run the same kernels on the same tables, so their group signals
must be bit-identical.  Two calls in a row share the scratch: the second,
with a smaller input (fewer rays, fewer bins and materials), must not see
anything of the first.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _static(fc, L, sp, mode, i0=None, S=None, s_bin=None):
    """Direct C-ABI call of fcat_spectral_static."""
    lib = fc.load()
    n = int(L.shape[0])
    Y = torch.full((sp.n_groups, n), float("nan"), dtype=torch.float32, device="cuda")
    cs, _keep = sp.c()
    ptr = lambda t: None if t is None else t.data_ptr()
    st = lib.fcat_spectral_static(L.data_ptr(), n, C.byref(cs), ptr(i0), ptr(S), ptr(s_bin), fc.MODES[mode],
                                  Y.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0, fc.fcat_last_error()
    return Y


def _inputs(cfg, n, seed):
    rng = np.random.default_rng(seed)
    M = cfg.spectral.n_mat
    L = rng.uniform(0.0, 40.0, size=(n, M)).astype(np.float32)
    L[rng.random(n) < 0.2] = 0.0                        # some misses
    L[:, rng.integers(0, M)] *= (rng.random(n) < 0.5)   # a material absent from half the rays
    i0 = rng.uniform(0.8, 1.2, n).astype(np.float32)
    S = rng.uniform(0.0, 0.1, n).astype(np.float32)
    s_bin = rng.uniform(0.5, 1.5, cfg.spectral.n_energy).astype(np.float32)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    return dev(L), dev(i0), dev(S), dev(s_bin)


@pytest.mark.parametrize("mode", ["plain", "split_bf16"])
def test_static_scratch_matches_workspace_call(fc, mode):
    big = synth.make_config(2)        # 8 materials, 200 bins, 8 groups
    small = synth.make_config(1)      # 6 materials, 32 bins, 1 group
    small.spectral.n_groups = 3
    small.spectral.group_of_bin = np.array([0] * 5 + [1] * 20 + [2] * 7, np.int32)
    for cfg, n, seed in ((big, 200_003, 1), (small, 1_001, 2)):
        sp = fc.upload(cfg, scatter=False, psf=False).spectral
        L, i0, S, s_bin = _inputs(cfg, n, seed)
        got = _static(fc, L, sp, mode, i0, S, s_bin)
        ref = fc.fcat_spectral(L, sp, i0=i0, S=S, s_bin=s_bin, mode=mode)
        torch.cuda.synchronize()
        print(f"{mode}: n {n}, E {cfg.spectral.n_energy}, M {cfg.spectral.n_mat}: "
              f"max |diff| {float((got - ref).abs().max()):.3e}")
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
        # without the optional inputs
        got = _static(fc, L, sp, mode)
        ref = fc.fcat_spectral(L, sp, mode=mode)
        assert torch.equal(got, ref)


def test_static_scratch_rejects_bad_arguments_before_launch(fc):
    lib = fc.load()
    sp = fc.upload(synth.make_config(1), scatter=False, psf=False).spectral
    cs, _keep = sp.c()
    assert lib.fcat_spectral_static(0x1000, -1, C.byref(cs), None, None, None, 0, 0x2000, None) == 1
    assert lib.fcat_spectral_static(0x1000, 10, C.byref(cs), None, None, None, 2, 0x2000, None) == 1
    assert lib.fcat_spectral_static(None, 10, C.byref(cs), None, None, None, 0, 0x2000, None) == 1
    assert lib.fcat_spectral_static(0x1000, 0, C.byref(cs), None, None, None, 0, None, None) == 0
