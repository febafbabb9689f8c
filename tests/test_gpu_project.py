"""End-to-end GPU parity of fcat_project with the FP64 oracle (plain FP32 mode).

Tolerance: 1e-5 relative per pixel (A-15 reading: |x - ref| / max(|ref|, 1e-12 max|ref|)).
Full-size configurations run in the benchmark's launch configuration (all
angles, default chunking); the oracle computes a sample of angles, which is
exact for a per-angle comparison because the optical spread does not couple
angles.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import rel_err

pytestmark = pytest.mark.gpu


def _check(out, cfg, angles, tol=1e-5, label=""):
    ref = oracle.project(cfg, angles)
    err = rel_err(out[angles], ref)
    print(f"{label}: angles {list(angles)[:6]}: max rel err {err.max():.3e}, rms {np.sqrt((err ** 2).mean()):.3e}")
    assert err.max() <= tol
    return err


def test_tiny_all_angles(fc):
    cfg = synth.make_config(1)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, list(range(45)), label="tiny")


def test_tiny_with_every_term(fc):
    """Flood map, scatter with per-bin scale, 3 groups with an uneven map,
    optical spread, explicit angles."""
    import torch
    cfg = synth.make_config(1)
    rng = np.random.default_rng(1)
    g, s = cfg.geometry, cfg.spectral
    g.angles = np.sort(rng.uniform(0, 2 * np.pi, size=g.n_angles))
    s.flood = rng.uniform(0.8, 1.2, size=(g.nv, g.nu)).astype(np.float32)
    s.n_groups = 3
    s.group_of_bin = np.array([0] * 5 + [1] * 20 + [2] * 7, np.int32)
    cfg.scatter = synth.scatter_blobs(rng, g.n_angles, g.nu, g.nv, (30, 60), (4, 8))
    cfg.scatter.s_bin = rng.uniform(0.5, 1.5, size=s.n_energy).astype(np.float32)
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 3, 15))
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, list(range(45)), label="tiny+all terms")
    # a small chunk (ragged last chunk) gives bit-identical results
    out7 = fc.fcat_project(pb, angles_per_chunk=7).cpu().numpy()
    np.testing.assert_array_equal(out7, out)
    # generic-k kernel path
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 3, 9))
    pb = fc.upload(cfg)
    out9 = fc.fcat_project(pb).cpu().numpy()
    _check(out9, cfg, [0, 13, 44], label="tiny k=9")
    del torch


def test_contrast_full_size(fc):
    """1024x1024x10 phantom, 200 bins, 1024x64 detector, 360 angles, scatter + 8x15x15 PSF."""
    cfg = synth.make_config(2)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    assert np.all(np.isfinite(out))
    _check(out, cfg, [0, 1, 90, 181, 300, 359], label="contrast")


def test_contrast_thick_slab_sampled(fc):
    cfg = synth.make_config(2, variant="z")
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, [0, 123, 359], label="contrast dz=1.5625")


def test_head_full_size_sampled(fc):
    """512x512x256 phantom, 120 bins, 1024x768 detector, 720 angles, scatter + PSF;
    eight full projections compared: the axis-parallel (0, 90 degrees) and
    diagonal (45, 135 degrees) directions, where crossings of two axes tie,
    and five others spread over the circle."""
    import torch
    cfg = synth.make_config(3)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb)
    sample = [0, 90, 180, 270, 333, 451, 600, 719]
    out_s = out[sample].cpu().numpy()
    del out, pb
    torch.cuda.empty_cache()
    ref = oracle.project(cfg, sample)
    err = rel_err(out_s, ref)
    print(f"head: max rel err {err.max():.3e}, rms {np.sqrt((err ** 2).mean()):.3e}")
    assert err.max() <= 1e-5


def test_repeatable_and_no_psf_sum(fc):
    cfg = synth.make_config(1)
    pb = fc.upload(cfg)
    a = fc.fcat_project(pb).cpu().numpy()
    for _ in range(3):
        np.testing.assert_array_equal(fc.fcat_project(pb).cpu().numpy(), a)


def test_degenerate_cases(fc):
    import torch
    cfg = synth.make_config(1)
    s = cfg.spectral
    # grid moved out of the cone: every ray misses, out = sum_e phi_e eta_e
    cfg.phantom.cz = 500.0
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    W = float(np.sum(s.phi.astype(np.float64) * s.eta.astype(np.float64)))
    assert np.all(np.abs(out - W) <= 1e-6 * W)
    # one pixel, one angle
    cfg = synth.make_config(1)
    cfg.geometry.nu, cfg.geometry.nv, cfg.geometry.n_angles = 1, 1, 1
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, [0], label="1x1x1")
    # one-voxel phantom, one energy bin
    cfg = synth.make_config(1)
    cfg.phantom.labels = np.ones((1, 1, 1), np.int8)
    cfg.phantom.dx = cfg.phantom.dy = cfg.phantom.dz = 5.0
    s.mu, s.phi, s.eta = s.mu[:, :1].copy(), s.phi[:1].copy(), s.eta[:1].copy()
    s.group_of_bin = np.zeros(1, np.int32)
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, list(range(45)), label="one voxel one bin")
    # a workspace that is too small is rejected and out stays untouched
    cfg = synth.make_config(2)
    cfg.phantom.labels = cfg.phantom.labels[:2].copy()
    pb = fc.upload(cfg)
    sentinel = torch.full((360, 64, 1024), 3.0, device="cuda")
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(fc.FcatError) as ei:
        fc.fcat_project(pb, out=sentinel, workspace=ws)
    assert ei.value.status == 2
    assert bool(torch.all(sentinel == 3.0))


def test_check_inputs(fc):
    import torch
    cfg = synth.make_config(1)
    pb = fc.upload(cfg)
    fc.fcat_check_inputs(pb)
    pb.phantom.labels[3, 4, 5] = 6                    # n_mat = 6: out of range
    with pytest.raises(fc.FcatError) as ei:
        fc.fcat_check_inputs(pb)
    assert ei.value.status == 3
    pb = fc.upload(cfg)
    pb.spectral.mu[2, 3] = float("nan")
    with pytest.raises(fc.FcatError) as ei:
        fc.fcat_check_inputs(pb)
    assert ei.value.status == 4
    # an out-of-range label never indexes out of bounds: it adds no path length
    pb = fc.upload(cfg)
    pb.phantom.labels[:, :, :] = torch.where(pb.phantom.labels == 2, torch.tensor(100, dtype=torch.int8,
                                             device="cuda"), pb.phantom.labels)
    out = fc.fcat_project(pb).cpu().numpy()
    cfg.spectral.mu[2] = 0.0
    ref = oracle.project(cfg, [0, 10])
    assert rel_err(out[[0, 10]], ref).max() <= 1e-5


def test_plain_tensor_entry(fc):
    """project() from plain device tensors equals fcat_project on the uploaded
    descriptors, bit for bit, and so the oracle: once bare, once with a flood
    map, scatter, 3 uneven groups and an optical spread."""
    cfg = synth.make_config(1)
    for full in (False, True):
        if full:
            rng = np.random.default_rng(2)
            g, s = cfg.geometry, cfg.spectral
            s.flood = rng.uniform(0.8, 1.2, size=(g.nv, g.nu)).astype(np.float32)
            s.n_groups = 3
            s.group_of_bin = np.array([0] * 6 + [1] * 18 + [2] * 8, np.int32)
            cfg.scatter = synth.scatter_blobs(rng, g.n_angles, g.nu, g.nv, (30, 60), (4, 8))
            cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 3, 15))
        pb = fc.upload(cfg)
        ref = fc.fcat_project(pb).cpu().numpy()
        ph, sp = pb.phantom, pb.spectral
        out = fc.project(pb.geometry, ph.labels, sp.mu, sp.phi, sp.eta,
                         scatter=None if pb.scatter is None else pb.scatter.maps,
                         psf=None if pb.psf is None else pb.psf.kernels, voxel=(ph.dx, ph.dy, ph.dz),
                         centre=(ph.cx, ph.cy, ph.cz), group_of_bin=sp.group_of_bin, flood=sp.flood)
        out = out.cpu().numpy()
        np.testing.assert_array_equal(out, ref)
        _check(out, cfg, [0, 22, 44], label=f"project() {'all terms' if full else 'bare'}")


def test_bit_identical_repeats_and_chunkings(fc):
    """Race check by repetition: ten calls on the contrast workload (walk with
    LDS material sums, LDS-tiled spread) and calls with other angle chunkings
    give bit-identical projections; so do repeated split-form calls."""
    import torch
    cfg = synth.make_config(2)
    pb = fc.upload(cfg)
    ref = fc.fcat_project(pb)
    buf = torch.empty_like(ref)
    for _ in range(10):
        fc.fcat_project(pb, out=buf)
        assert torch.equal(buf, ref)
    for ch in (7, 90):
        assert torch.equal(fc.fcat_project(pb, angles_per_chunk=ch), ref)
    sref = fc.fcat_project(pb, mode="split_bf16")
    for _ in range(3):
        assert torch.equal(fc.fcat_project(pb, mode="split_bf16", out=buf), sref)


def test_thin_slab(fc):
    """A thin slab (a band of a few detector rows of shadow: the 16 x 4 pixel
    wavefront tiles) with a flood map, scatter, 3 groups and an optical
    spread, all angles against the oracle, with and without the spread;
    ragged angle chunks give the same bits."""
    rng = np.random.default_rng(7)
    cfg = synth.make_config(1)
    ph, g, s = cfg.phantom, cfg.geometry, cfg.spectral
    ph.labels = ph.labels[6:9].copy()                 # 3 slices of 1 mm: a band of ~4.5 detector rows
    s.flood = rng.uniform(0.8, 1.2, size=(g.nv, g.nu)).astype(np.float32)
    s.n_groups = 3
    s.group_of_bin = np.array([0] * 9 + [1] * 13 + [2] * 10, np.int32)
    cfg.scatter = synth.scatter_blobs(rng, g.n_angles, g.nu, g.nv, (30, 60), (4, 8))
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 3, 15))
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, list(range(45)), label="thin slab")
    np.testing.assert_array_equal(fc.fcat_project(pb, angles_per_chunk=7).cpu().numpy(), out)
    cfg.psf = None
    pb = fc.upload(cfg)
    out = fc.fcat_project(pb).cpu().numpy()
    _check(out, cfg, [0, 11, 44], label="thin slab, no spread")
