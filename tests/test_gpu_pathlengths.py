"""GPU parity of the ray traversal (per-material path lengths) with the FP64 oracle.

Sec. II.F: a projection is the line integral of the attenuation along the
ray; Sec. II.C: labelled phantom.  The HIP traversal works in FP32 distance
from an FP64 entry point, so its error is a few FP32 ulps of the chord per
material transition; the bound used here is 3e-5 mm + 1e-6 of the chord.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Geometry, Phantom

pytestmark = pytest.mark.gpu


def _tol(Lref):
    total = Lref.sum(axis=-1, keepdims=True)
    return 3e-5 + 1e-6 * total


def _upload_geo_phantom(fc, geo, ph):
    import torch
    ang = None if geo.angles is None else torch.as_tensor(np.asarray(geo.angles, np.float64), device="cuda")
    g = fc.Geometry(geo.sid, geo.sdd, geo.nu, geo.nv, geo.du, geo.dv, geo.n_angles, geo.off_u, geo.off_v, ang)
    p = fc.Phantom(torch.as_tensor(ph.labels, device="cuda"), ph.dx, ph.dy, ph.dz, ph.cx, ph.cy, ph.cz)
    return fc.Problem(g, p, None)


def test_tiny_config_all_angles(fc):
    cfg = synth.make_config(1)
    pb = _upload_geo_phantom(fc, cfg.geometry, cfg.phantom)
    M = cfg.spectral.n_mat
    L = fc.fcat_pathlengths(pb, M).cpu().numpy()
    Lref = oracle.pathlengths(cfg.geometry, cfg.phantom, M, range(cfg.geometry.n_angles))
    err = np.abs(L - Lref)
    print(f"tiny: max |dL| = {err.max():.3e} mm, max chord {Lref.sum(-1).max():.2f}")
    assert np.all(err <= _tol(Lref))
    assert (Lref.sum(-1) > 0).mean() > 0.5


@pytest.mark.parametrize("seed,n_mat", [(0, 5), (1, 13), (2, 20), (3, 32)])
def test_random_phantoms_ragged_detector(fc, seed, n_mat):
    """Random labels, anisotropic voxels, off-centre grid, explicit angles and a
    detector whose width is not a multiple of the 64-lane wavefront."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = rng.integers(5, 40, size=3)
    labels = synth.random_phantom(rng, int(nx), int(ny), int(nz), n_mat)
    h = rng.uniform(0.3, 1.5, size=3)
    ph = Phantom(dx=h[0], dy=h[1], dz=h[2], labels=labels,
                 cx=rng.uniform(-3, 3), cy=rng.uniform(-3, 3), cz=rng.uniform(-2, 2))
    A = 7
    geo = Geometry(sid=rng.uniform(80, 200), sdd=rng.uniform(250, 400), nu=int(rng.integers(65, 200)),
                   nv=int(rng.integers(3, 12)), du=rng.uniform(0.3, 1.2), dv=rng.uniform(0.3, 1.2),
                   n_angles=A, off_u=rng.uniform(-2, 2), off_v=rng.uniform(-1, 1),
                   angles=rng.uniform(0, 2 * np.pi, size=A))
    pb = _upload_geo_phantom(fc, geo, ph)
    L = fc.fcat_pathlengths(pb, n_mat, 2, 6).cpu().numpy()
    Lref = oracle.pathlengths(geo, ph, n_mat, [2, 3, 4, 5])
    err = np.abs(L - Lref)
    print(f"seed {seed} M={n_mat} grid {nx}x{ny}x{nz} det {geo.nu}x{geo.nv}: max |dL| {err.max():.3e}")
    assert np.all(err <= _tol(Lref))


def test_contrast_phantom_sampled_angles(fc):
    cfg = synth.make_config(2)
    pb = _upload_geo_phantom(fc, cfg.geometry, cfg.phantom)
    M = cfg.spectral.n_mat
    for a in (0, 37, 359):
        L = fc.fcat_pathlengths(pb, M, a, a + 1).cpu().numpy()
        Lref = oracle.pathlengths(cfg.geometry, cfg.phantom, M, [a])
        err = np.abs(L - Lref)
        print(f"contrast angle {a}: max |dL| {err.max():.3e}, hit fraction {(Lref.sum(-1) > 0).mean():.3f}")
        assert np.all(err <= _tol(Lref))


def test_uniform_volume_total_is_chord(fc):
    """Any labelling: sum_m L_m is the chord of the grid, whatever the labels."""
    rng = np.random.default_rng(9)
    labels = synth.random_phantom(rng, 50, 40, 30, 6)
    ph = Phantom(dx=0.7, dy=0.9, dz=0.8, labels=labels)
    ones = Phantom(dx=0.7, dy=0.9, dz=0.8, labels=np.ones_like(labels))
    geo = Geometry(sid=300.0, sdd=450.0, nu=130, nv=33, du=0.6, dv=0.6, n_angles=5)
    L = fc.fcat_pathlengths(_upload_geo_phantom(fc, geo, ph), 6).cpu().numpy()
    L1 = fc.fcat_pathlengths(_upload_geo_phantom(fc, geo, ones), 6).cpu().numpy()
    assert np.all(L1[..., [0, 2, 3, 4, 5]] == 0)
    np.testing.assert_allclose(L.sum(-1), L1[..., 1], rtol=2e-6, atol=3e-5)


def test_axis_aligned_and_parallel_rays(fc):
    """Angle 0 puts the central detector row in the z = 0 plane between two
    voxel layers (ties are resolved to the + side) and rays parallel to x."""
    labels = np.zeros((4, 6, 6), np.int8)
    labels[2] = 1                                   # z in [0, 1): the + side of z = 0
    labels[1] = 2
    ph = Phantom(dx=1.0, dy=1.0, dz=1.0, labels=labels)
    geo = Geometry(sid=100.0, sdd=150.0, nu=5, nv=3, du=0.5, dv=0.5, n_angles=4)
    pb = _upload_geo_phantom(fc, geo, ph)
    L = fc.fcat_pathlengths(pb, 3).cpu().numpy()
    Lref = oracle.pathlengths(geo, ph, 3, range(4))
    np.testing.assert_allclose(L, Lref, rtol=1e-6, atol=3e-5)
    assert Lref[0, 1, 2, 1] > 5.9                     # central ray runs inside layer z in [0, 1)


@pytest.mark.parametrize("seed,shape,blocks", [(0, (61, 45, 27), (3, 20)), (1, (61, 45, 27), (3, 20)),
                                               (2, (97, 83, 53), (16, 48))])
def test_blocky_phantom_brick_walk(fc, seed, shape, blocks):
    """Piecewise-constant blocks of random sizes (with the larger blocks many
    bricks are uniform, others mixed, partial bricks at the grid edge) with
    random noise patches: the two-level walk must match the exact path
    lengths everywhere."""
    rng = np.random.default_rng(40 + seed)
    nx, ny, nz = shape                              # not multiples of the brick edge
    labels = np.zeros((nz, ny, nx), np.int8)
    for _ in range(25):
        x0, y0, z0 = rng.integers(0, [nx, ny, nz])
        sx, sy, sz = rng.integers(*blocks, size=3)
        labels[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = rng.integers(0, 7)
    for _ in range(6):
        x0, y0, z0 = rng.integers(0, [nx - 4, ny - 4, nz - 4])
        labels[z0:z0 + 4, y0:y0 + 4, x0:x0 + 4] = rng.integers(0, 7, size=(4, 4, 4))
    ph = Phantom(dx=0.5, dy=0.5, dz=0.5, labels=labels, cx=0.3, cy=-0.2, cz=0.1)
    geo = Geometry(sid=150.0, sdd=250.0, nu=157, nv=61, du=0.35, dv=0.35, n_angles=12)
    pb = _upload_geo_phantom(fc, geo, ph)
    L = fc.fcat_pathlengths(pb, 7).cpu().numpy()
    Lref = oracle.pathlengths(geo, ph, 7, range(12))
    err = np.abs(L - Lref)
    print(f"blocky seed {seed}: max |dL| {err.max():.3e}")
    assert np.all(err <= _tol(Lref))


@pytest.mark.parametrize("offset", [(16, 16, 16), (17, 5, 30)])
def test_background_box(fc, offset):
    """A mixed object in a uniform background away from the grid's corner: the
    walk runs only inside the brick-aligned box around the object and charges
    the rest of each ray to the background in one sum.  Angle 0 runs rays
    exactly along voxel and box planes (ties), the others cross the box's
    faces and corners at general angles; the exact path lengths must hold
    everywhere.  (Angles of 90, 180 or 270 degrees are left out: there the
    rounded cosine or sine tilts the central rays by about 1e-14 mm against a
    voxel plane, and which voxel such a ray is in is decided below the FP64
    resolution of the oracle's midpoint indices; an exact rational evaluation
    of those rays agrees with the walk.)"""
    rng = np.random.default_rng(77)
    nx, ny, nz = 70, 66, 50
    labels = np.full((nz, ny, nx), 3, np.int8)
    x0, y0, z0 = offset
    labels[z0:z0 + 9, y0:y0 + 12, x0:x0 + 20] = rng.integers(0, 5, size=(9, 12, 20))
    ph = Phantom(dx=1.0, dy=1.0, dz=1.0, labels=labels)
    angles = np.array([0.0, 0.31, 0.785, 1.1, 2.0, 2.9, 3.6, 4.4, 5.5])
    geo = Geometry(sid=200.0, sdd=320.0, nu=141, nv=97, du=0.8, dv=0.8, n_angles=len(angles), angles=angles)
    pb = _upload_geo_phantom(fc, geo, ph)
    L = fc.fcat_pathlengths(pb, 5).cpu().numpy()
    Lref = oracle.pathlengths(geo, ph, 5, range(len(angles)))
    err = np.abs(L - Lref)
    print(f"background box {offset}: max |dL| {err.max():.3e}")
    assert np.all(err <= _tol(Lref))
    np.testing.assert_allclose(L.sum(-1), Lref.sum(-1), rtol=2e-6, atol=3e-5)
