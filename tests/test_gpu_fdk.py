"""GPU parity of the FDK reconstruction (Sec. II.G) with the FP64 oracle.

Tolerances, from the FP32 arithmetic of the kernels:
* ramp filter: a row output sums nu/2 products in FP32, bounded by
  2e-5 max|p| / tau (the filter's gain is of order 1 / tau);
* back-projection: the detector position of a voxel is computed in FP32
  (1e-5 pixel) and the sum runs over the angles in FP32, giving 2e-5 of the
  largest value of the volume;
* the whole reconstruction: the two added, 5e-5 of the largest value.
The oracle always takes the same float32 projections as the kernels.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import fdk as ofdk

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _geom(fc, g, angles=None):
    return fc.Geometry(sid=g.sid, sdd=g.sdd, nu=g.nu, nv=g.nv, du=g.du, dv=g.dv, n_angles=g.n_angles,
                       off_u=g.off_u, off_v=g.off_v, angles=None if angles is None else _dev(angles))


@pytest.mark.parametrize("nu,nv", [(128, 16), (157, 13), (1024, 3)])
def test_filter_parity(fc, nu, nv):
    rng = np.random.default_rng(nu)
    g = synth.Geometry(sid=900.0, sdd=1400.0, nu=nu, nv=nv, du=0.4, dv=0.5, n_angles=3, off_u=1.3, off_v=-0.7)
    p = rng.uniform(0.0, 3.0, (3, nv, nu)).astype(np.float32)
    got = fc.fcat_fdk_filter(_geom(fc, g), _dev(p)).cpu().numpy()
    ref = ofdk.filter_projections(p, g)
    tau = g.du * g.sid / g.sdd
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(p).max() / tau


def test_backprojection_parity(fc):
    rng = np.random.default_rng(7)
    g = synth.Geometry(sid=400.0, sdd=650.0, nu=96, nv=20, du=0.8, dv=0.8, n_angles=40, off_u=-1.1, off_v=0.6)
    filt = (ofdk.filter_projections(rng.uniform(0.0, 2.0, (40, 20, 96)), g)).astype(np.float32)
    grid = synth.Grid(nx=70, ny=45, nz=11, dx=0.9, dy=1.1, dz=0.7, cx=2.0, cy=-3.0, cz=0.5)
    vol = fc.fcat_fdk_backproject(_geom(fc, g), _dev(filt), grid).cpu().numpy()
    ref = ofdk.backproject(filt, g, ofdk.grid_points(grid)).reshape(vol.shape)
    assert np.abs(vol - ref).max() <= 2e-5 * np.abs(ref).max()
    # explicit, uneven angles; an angle sub-range accumulated onto a volume
    ang = np.sort(rng.uniform(0.0, 2 * np.pi, 40))
    g2 = synth.Geometry(**{**g.__dict__, "angles": ang})
    part = fc.fcat_fdk_backproject(_geom(fc, g2, ang), _dev(filt[:25]), grid)
    fc.fcat_fdk_backproject(_geom(fc, g2, ang), _dev(filt[25:]), grid, a_begin=25, volume=part, accumulate=True)
    ref2 = ofdk.backproject(filt, g2, ofdk.grid_points(grid)).reshape(vol.shape)
    assert np.abs(part.cpu().numpy() - ref2).max() <= 2e-5 * np.abs(ref2).max()


def test_fdk_tiny_parity_and_chunks(fc, orc):
    # monoenergetic projections of the tiny phantom by the projector oracle
    cfg = synth.make_config(1)
    g, s = cfg.geometry, cfg.spectral
    L = orc.pathlengths(g, cfg.phantom, s.n_mat, list(range(g.n_angles)))
    proj = (L @ s.mu[:, 10].astype(np.float64)).astype(np.float32)
    grid = synth.Grid(nx=64, ny=64, nz=8, dx=1.0, dy=1.0, dz=1.0)
    fg = _geom(fc, g)
    vol = fc.fcat_fdk(fg, _dev(proj), grid).cpu().numpy()
    ref = ofdk.fdk(proj, g, grid)
    err = np.abs(vol - ref).max() / np.abs(ref).max()
    print(f"tiny fdk: max |err| / max|f| = {err:.2e}")
    assert err <= 5e-5
    vol7 = fc.fcat_fdk(fg, _dev(proj), grid, angles_per_chunk=7).cpu().numpy()
    assert np.abs(vol7 - vol).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("nu,nv", [(1, 5), (6, 1), (33, 9)])
def test_fdk_off_detector_and_degenerate_detectors(fc, nu, nv):
    """The whole reconstruction back-projects zero-padded filtered rows: a
    grid far wider and taller than the field of view (voxels off every edge
    of the detector), one-column and one-row detectors, and 37 slices (z
    blocks of 13, 13 and 11); against the oracle, against the filter and
    dense back-projection entry points, and in chunks of 5 angles."""
    rng = np.random.default_rng(nu * 10 + nv)
    g = synth.Geometry(sid=300.0, sdd=450.0, nu=nu, nv=nv, du=1.2, dv=1.1, n_angles=24, off_u=0.3, off_v=-0.2)
    proj = rng.uniform(0.0, 2.0, (24, nv, nu)).astype(np.float32)
    grid = synth.Grid(nx=29, ny=23, nz=37, dx=1.5, dy=1.5, dz=0.9, cx=1.0, cy=-2.0, cz=0.4)
    fg = _geom(fc, g)
    vol = fc.fcat_fdk(fg, _dev(proj), grid).cpu().numpy()
    ref = ofdk.fdk(proj, g, grid)
    scale = np.abs(ref).max()
    assert scale > 0 and np.any(ref == 0.0)          # some voxels see no detector at all
    err = np.abs(vol - ref).max() / scale
    dense = fc.fcat_fdk_backproject(fg, fc.fcat_fdk_filter(fg, _dev(proj)), grid).cpu().numpy()
    d_err = np.abs(vol - dense).max() / scale
    vol5 = fc.fcat_fdk(fg, _dev(proj), grid, angles_per_chunk=5).cpu().numpy()
    c_err = np.abs(vol5 - vol).max() / scale
    print(f"nu {nu} nv {nv}: vs oracle {err:.2e}, vs dense {d_err:.2e}, chunks {c_err:.2e}")
    assert err <= 5e-5 and d_err <= 5e-6 and c_err <= 5e-6


def test_fdk_contrast_sampled(fc, orc):
    # the contrast workload: 360 x 64 x 1024 projections into its 1024 x 1024 x 10
    # grid in one call; 1,500 sampled voxels against the oracle
    import torch
    cfg = synth.make_config(2)
    g, s, ph = cfg.geometry, cfg.spectral, cfg.phantom
    L = orc.pathlengths(g, ph, s.n_mat, list(range(g.n_angles)))
    proj = (L @ s.mu[:, 60].astype(np.float64)).astype(np.float32)
    del L
    grid = synth.Grid(nx=ph.nx, ny=ph.ny, nz=ph.nz, dx=ph.dx, dy=ph.dy, dz=ph.dz)
    vol = fc.fcat_fdk(_geom(fc, g), _dev(proj), grid)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, grid.nz, 1500), rng.integers(0, grid.ny, 1500),
                    rng.integers(0, grid.nx, 1500)], axis=1)
    got = vol[tuple(torch.as_tensor(idx.T).cuda())].cpu().numpy()
    filt = ofdk.filter_projections(proj, g)
    ref = ofdk.backproject(filt, g, ofdk.grid_points(grid, idx))
    scale = np.abs(ref).max()
    print(f"contrast fdk: max |err| / max|f| = {np.abs(got - ref).max() / scale:.2e}")
    assert np.abs(got - ref).max() <= 5e-5 * scale


def test_fdk_reconstructs_the_projector_cylinder(fc):
    # the GPU projector's own monoenergetic projections of a water cylinder
    # (one energy bin, no scatter or spread) reconstruct to mu inside
    import torch
    h = 0.5
    labels = synth.cylinder_phantom(96, 96, 12, h, h, 20.0, [])
    ph = synth.Phantom(dx=h, dy=h, dz=h, labels=labels)
    g = synth.Geometry(sid=600.0, sdd=900.0, nu=128, nv=12, du=0.6, dv=0.6, n_angles=180)
    mu = np.array([[0.0], [0.02]], np.float32)
    spec = synth.Spectral(energies=np.array([60.0]), mu=mu, phi=np.ones(1, np.float32), eta=np.ones(1, np.float32),
                          n_groups=1, group_of_bin=np.zeros(1, np.int32))
    cfg = synth.Config("cyl", g, ph, spec)
    pb = fc.upload(cfg)
    proj = fc.fcat_projections(pb, None)
    grid = synth.Grid(nx=48, ny=48, nz=1, dx=1.0, dy=1.0, dz=0.5, cz=0.25)
    vol = fc.fcat_fdk(pb.geometry, proj, grid).cpu().numpy()[0]
    x, y, _ = ofdk.voxel_centres(grid)
    X, Y = np.meshgrid(x, y, indexing="xy")
    inside = vol[np.hypot(X, Y) < 17.0]
    outside = vol[(np.hypot(X, Y) > 22.5) & (np.hypot(X, Y) < 25.0)]   # inside the 25.6 mm field of view
    # mean within 1.5 %; the staircase of the 0.5 mm labels and 180 views leave
    # a few per cent of local ripple
    assert abs(inside.mean() / 0.02 - 1.0) < 0.015 and inside.std() / 0.02 < 0.03
    assert abs(outside.mean()) < 0.02 * 0.02
    del torch
