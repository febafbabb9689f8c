"""Pins of the oracle's image projector A and its transpose A^T.

A f integrates a real-valued voxel image along each source-to-pixel ray
(the Sec. II.F line integral over an image, as an iterative reconstruction
of Sec. II.G uses it); A^T spreads each ray's value back over the voxels it
crosses, weighted by the length inside each.  Pinned by: the closed-form
chord through the grid for a uniform image; an independent midpoint-rule
sampler on tiny random images; the labelled projector's path lengths for an
indicator image; the adjoint identity <A f, y> = <f, A^T y>; and a single
ray's back-projection holding exactly its chord, on exactly its voxels.
"""
import numpy as np
import pytest

import oracle
import synth


def _setup(nx=6, ny=5, nz=4, A=5, nu=9, nv=7, seed=0):
    rng = np.random.default_rng(seed)
    geo = synth.Geometry(sid=40.0, sdd=70.0, nu=nu, nv=nv, du=1.3, dv=1.1, n_angles=A, off_u=0.17, off_v=-0.23)
    grid = synth.Grid(nx=nx, ny=ny, nz=nz, dx=1.5, dy=1.2, dz=1.7, cx=0.3, cy=-0.4, cz=0.2)
    return rng, geo, grid


def _rays(geo):
    """Source and pixel-centre points of every ray, [A][nv][nu][3], from the conventions."""
    th = geo.angle_values()
    pu = (np.arange(geo.nu) - (geo.nu - 1) / 2) * geo.du + geo.off_u
    pv = (np.arange(geo.nv) - (geo.nv - 1) / 2) * geo.dv + geo.off_v
    S, D = [], []
    for t in th:
        c, s = np.cos(t), np.sin(t)
        src = np.array([geo.sid * c, geo.sid * s, 0.0])
        cen = -(geo.sdd - geo.sid) * np.array([c, s, 0.0])
        u = np.array([-s, c, 0.0])
        dst = cen[None, None, :] + pu[None, :, None] * u[None, None, :] + pv[:, None, None] * np.array([0, 0, 1.0])
        S.append(np.broadcast_to(src, dst.shape))
        D.append(dst)
    return np.array(S), np.array(D)


def _box(grid):
    n = np.array([grid.nx, grid.ny, grid.nz], float)
    h = np.array([grid.dx, grid.dy, grid.dz])
    lo = np.array([grid.cx, grid.cy, grid.cz]) - n * h / 2
    return lo, lo + n * h, n, h


def test_uniform_image_gives_the_chord():
    _, geo, grid = _setup()
    f = np.ones((grid.nz, grid.ny, grid.nx))
    got = oracle.forward_image(geo, grid, f, range(geo.n_angles))
    S, D = _rays(geo)
    lo, hi, _, _ = _box(grid)
    d = D - S
    with np.errstate(divide="ignore", invalid="ignore"):
        a0, a1 = (lo - S) / d, (hi - S) / d
        amin = np.maximum(0.0, np.nanmax(np.minimum(a0, a1), -1))
        amax = np.minimum(1.0, np.nanmin(np.maximum(a0, a1), -1))
    chord = np.maximum(amax - amin, 0.0) * np.linalg.norm(d, axis=-1)
    assert (chord > 0).mean() > 0.3
    np.testing.assert_allclose(got, chord, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [1, 2])
def test_random_image_against_midpoint_sampling(seed):
    rng, geo, grid = _setup(seed=seed)
    f = rng.uniform(-1.0, 2.0, size=(grid.nz, grid.ny, grid.nx))
    got = oracle.forward_image(geo, grid, f, range(geo.n_angles))
    S, D = _rays(geo)
    lo, hi, n, h = _box(grid)
    steps = 20000
    t = (np.arange(steps) + 0.5) / steps
    ref = np.zeros(got.shape)
    bound = np.zeros(got.shape)
    for idx in np.ndindex(got.shape):
        s, dd = S[idx], D[idx] - S[idx]
        pts = s[None, :] + t[:, None] * dd[None, :]
        q = np.floor((pts - lo) / h)
        inside = np.all((q >= 0) & (q < n), axis=1)
        qi = q[inside].astype(int)
        vals = f[qi[:, 2], qi[:, 1], qi[:, 0]]
        step = np.linalg.norm(dd) / steps
        ref[idx] = vals.sum() * step
        changes = 2 + (np.abs(np.diff(qi, axis=0)).sum() if len(qi) else 0)
        bound[idx] = step * changes * np.abs(f).max()
    assert np.all(np.abs(got - ref) <= bound + 1e-12)


def test_indicator_image_gives_the_labelled_path_lengths():
    rng, geo, grid = _setup(seed=3)
    labels = rng.integers(0, 4, size=(grid.nz, grid.ny, grid.nx)).astype(np.int8)
    ph = synth.Phantom(dx=grid.dx, dy=grid.dy, dz=grid.dz, labels=labels, cx=grid.cx, cy=grid.cy, cz=grid.cz)
    L = oracle.pathlengths(geo, ph, 4, range(geo.n_angles))
    for m in range(4):
        got = oracle.forward_image(geo, grid, (labels == m).astype(float), range(geo.n_angles))
        np.testing.assert_allclose(got, L[..., m], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [4, 5])
def test_adjoint_identity(seed):
    rng, geo, grid = _setup(nx=11, ny=9, nz=7, A=7, seed=seed)
    f = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    y = rng.normal(size=(geo.n_angles, geo.nv, geo.nu))
    Af = oracle.forward_image(geo, grid, f, range(geo.n_angles))
    ATy = oracle.backproject_image(geo, grid, y, range(geo.n_angles))
    lhs, rhs = float((Af * y).sum()), float((f * ATy).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.abs(Af * y).sum())


def test_one_ray_back_projects_its_chord_onto_its_voxels():
    _, geo, grid = _setup()
    ones = np.ones((grid.nz, grid.ny, grid.nx))
    chord = oracle.forward_image(geo, grid, ones, range(geo.n_angles))
    a, iv, iu = 2, 3, 4
    assert chord[a, iv, iu] > 0
    y = np.zeros((geo.n_angles, geo.nv, geo.nu))
    y[a, iv, iu] = 1.0
    img = oracle.backproject_image(geo, grid, y, range(geo.n_angles))
    assert img.sum() == pytest.approx(chord[a, iv, iu], rel=1e-12)
    # exactly the voxels a fine midpoint sampling of the ray visits (up to
    # voxels it only grazes, whose share of the chord is tiny)
    S, D = _rays(geo)
    lo, hi, n, h = _box(grid)
    t = (np.arange(200000) + 0.5) / 200000
    pts = S[a, iv, iu][None, :] + t[:, None] * (D[a, iv, iu] - S[a, iv, iu])[None, :]
    q = np.floor((pts - lo) / h)
    q = q[np.all((q >= 0) & (q < n), axis=1)].astype(int)
    seen = np.zeros(img.shape, bool)
    seen[q[:, 2], q[:, 1], q[:, 0]] = True
    assert np.all(img[~seen] < 1e-4 * chord[a, iv, iu]) and np.all(img[seen] > 0)
