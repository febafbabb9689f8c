"""GPU parity of the dose estimate (Sec. II.H, Eqs. 6-7) with the FP64 oracle.

Tolerance 1e-5 relative per energy bin and for D_p: path lengths carry
~1e-6 relative error, P and 1 - exp(-P) a few FP32 ulp; every sum runs in
FP64.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dose as od

pytestmark = pytest.mark.gpu


def _dose_inputs(cfg, rng):
    s = cfg.spectral
    e_ref = 30.0 if s.energy_unit == "keV" else 1.0
    ratio = synth.energy_absorption_ratio(rng, s.energies, e_ref)
    energy = s.energies.astype(np.float32)
    mass = synth.phantom_mass_kg(cfg.phantom, synth.material_densities(s.material_names))
    return energy, ratio, mass


def _oracle_dose(cfg, angles, energy, ratio, mass):
    s, g = cfg.spectral, cfg.geometry
    L = oracle.pathlengths(g, cfg.phantom, s.n_mat, angles).reshape(-1, s.n_mat)
    hit = L.any(axis=1)
    return od.dose_per_particle(L[hit], s.mu, energy, ratio, s.phi, mass, n_rays=L.shape[0])


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def test_dose_tiny_all_angles(fc):
    rng = np.random.default_rng(61)
    cfg = synth.make_config(1)
    energy, ratio, mass = _dose_inputs(cfg, rng)
    pb = fc.upload(cfg)
    D0, Dp = fc.fcat_dose(pb, _dev(energy), _dev(ratio), mass)
    D0 = D0.cpu().numpy()
    ref0, refp = _oracle_dose(cfg, list(range(cfg.geometry.n_angles)), energy, ratio, mass)
    err = np.abs(D0 / ref0 - 1)
    print(f"tiny: max rel err per bin {err.max():.2e}, Dp {abs(float(Dp) / refp - 1):.2e}")
    assert err.max() <= 1e-5 and abs(float(Dp) / refp - 1) <= 1e-5
    # an angle sub-range, and a small chunk with a ragged end: same sums up to FP64 order
    D0s, _ = fc.fcat_dose(pb, _dev(energy), _dev(ratio), mass, a_begin=7, a_end=30, angles_per_chunk=4)
    ref_s, _ = _oracle_dose(cfg, list(range(7, 30)), energy, ratio, mass)
    assert np.abs(D0s.cpu().numpy() / ref_s - 1).max() <= 1e-5


def test_dose_contrast_full(fc):
    # the contrast workload: 360 angles x 1024 x 64 rays, 8 materials, 200 bins
    rng = np.random.default_rng(62)
    cfg = synth.make_config(2)
    energy, ratio, mass = _dose_inputs(cfg, rng)
    pb = fc.upload(cfg)
    D0, Dp = fc.fcat_dose(pb, _dev(energy), _dev(ratio), mass)
    D0 = D0.cpu().numpy()
    ref0, refp = _oracle_dose(cfg, list(range(cfg.geometry.n_angles)), energy, ratio, mass)
    err = np.abs(D0 / ref0 - 1)
    print(f"contrast: max rel err per bin {err.max():.2e}, Dp {abs(float(Dp) / refp - 1):.2e}")
    assert err.max() <= 1e-5 and abs(float(Dp) / refp - 1) <= 1e-5


@pytest.mark.parametrize("n_bins", [1, 37, 300])
def test_dose_bin_counts(fc, n_bins):
    """Bin counts that do not fill the workgroups (1, an odd 37, 300), whose
    work is split in stripes of rays; all angles of the tiny case."""
    rng = np.random.default_rng(65 + n_bins)
    cfg = synth.make_config(1)
    s = cfg.spectral
    idx = np.arange(n_bins) % s.mu.shape[1]
    s.energies = np.asarray(s.energies)[idx].copy()
    s.mu = s.mu[:, idx].copy()
    s.phi = s.phi[idx].copy()
    s.eta = s.eta[idx].copy()
    s.n_groups = 1
    s.group_of_bin = np.zeros(n_bins, np.int32)
    energy, ratio, mass = _dose_inputs(cfg, rng)
    pb = fc.upload(cfg, scatter=False, psf=False)
    D0, Dp = fc.fcat_dose(pb, _dev(energy), _dev(ratio), mass)
    D0 = D0.cpu().numpy()
    ref0, refp = _oracle_dose(cfg, list(range(cfg.geometry.n_angles)), energy, ratio, mass)
    err = np.abs(D0 / ref0 - 1)
    print(f"{n_bins} bins: max rel err per bin {err.max():.2e}, Dp {abs(float(Dp) / refp - 1):.2e}")
    assert err.max() <= 1e-5 and abs(float(Dp) / refp - 1) <= 1e-5


def test_dose_all_rays_miss(fc):
    # detector shifted far off the phantom: every ray misses, the dose is exactly 0
    rng = np.random.default_rng(63)
    cfg = synth.make_config(1)
    cfg.geometry.off_v = 500.0
    energy, ratio, mass = _dose_inputs(cfg, rng)
    pb = fc.upload(cfg)
    D0, Dp = fc.fcat_dose(pb, _dev(energy), _dev(ratio), mass)
    assert np.all(D0.cpu().numpy() == 0.0) and float(Dp) == 0.0


def test_dose_rejects_bad_arguments(fc):
    rng = np.random.default_rng(64)
    cfg = synth.make_config(1)
    energy, ratio, _ = _dose_inputs(cfg, rng)
    pb = fc.upload(cfg)
    with pytest.raises(fc.FcatError):
        fc.fcat_dose(pb, _dev(energy), _dev(ratio), 0.0)
    with pytest.raises(fc.FcatError):
        fc.fcat_dose(pb, _dev(energy), _dev(ratio), 1.0, a_begin=5, a_end=5)
