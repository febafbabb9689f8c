"""Pins of the FDK oracle (oracle/fdk.py).

Expected values: the frequency response of the Ram-Lak kernel (|f| up to
the Nyquist frequency, zero at DC); closed-form projections of uniform
cylinders, whose reconstruction must give the attenuation inside and zero
outside; the projector oracle's own projections of a voxelised cylinder.
Sec. II.G (reconstruction with FDK); Feldkamp, Davis and Kress (1984).
"""
import math

import numpy as np
import pytest

import synth
from oracle import fdk


def test_ramp_kernel_frequency_response():
    # the DTFT of tau h(k tau) is |f| for |f| <= 1 / (2 tau): zero at DC, 1/(2 tau) at Nyquist
    tau, n = 0.25, 4001
    h = fdk.ramp_kernel(n, tau)
    k = np.arange(-(n - 1), n)
    for f in (0.0, 0.1, 0.5, 1.0, 1.5, 2.0):
        H = float(np.sum(h * np.cos(2 * math.pi * f * k * tau)))
        # truncation of the 1/k^2 tail leaves an error below 2 / (pi^2 tau n)
        assert abs(H - abs(f)) < 2.0 / (math.pi ** 2 * tau * n) + 1e-12, (f, H)
    # taps: 1/(4 tau) at 0, zero at even offsets, negative at odd ones
    c = n - 1
    assert abs(h[c] - 1.0 / (4 * tau)) < 1e-15
    assert np.all(h[c + 2::2] == 0.0) and np.all(h[c + 1::2] < 0.0)


def _cylinder_projections(g, mu, R, x0, y0, half_h, z0=0.0):
    """mu times the exact chord of every ray through the cylinder
    (x - x0)^2 + (y - y0)^2 <= R^2, |z - z0| <= half_h."""
    out = np.zeros((g.n_angles, g.nv, g.nu))
    for ai, b in enumerate(g.angle_values()):
        cb, sb = math.cos(b), math.sin(b)
        src = np.array([g.sid * cb, g.sid * sb, 0.0])
        ctr = -(g.sdd - g.sid) * np.array([cb, sb, 0.0])
        eu, ev = np.array([-sb, cb, 0.0]), np.array([0.0, 0.0, 1.0])
        uu = (np.arange(g.nu) - (g.nu - 1) / 2) * g.du + g.off_u
        vv = (np.arange(g.nv) - (g.nv - 1) / 2) * g.dv + g.off_v
        pix = ctr[None, None] + uu[None, :, None] * eu + vv[:, None, None] * ev
        d = pix - src
        sx, sy = src[0] - x0, src[1] - y0
        A = d[..., 0] ** 2 + d[..., 1] ** 2
        B = 2 * (sx * d[..., 0] + sy * d[..., 1])
        C = sx * sx + sy * sy - R * R
        disc = B * B - 4 * A * C
        ok = disc > 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t1, t2 = (-B - sq) / (2 * A), (-B + sq) / (2 * A)
        with np.errstate(divide="ignore", invalid="ignore"):
            z1 = np.where(d[..., 2] != 0, (z0 - half_h - src[2]) / d[..., 2], -np.inf)
            z2 = np.where(d[..., 2] != 0, (z0 + half_h - src[2]) / d[..., 2], np.inf)
        lo, hi = np.minimum(z1, z2), np.maximum(z1, z2)
        t1, t2 = np.maximum(np.maximum(t1, lo), 0.0), np.minimum(np.minimum(t2, hi), 1.0)
        out[ai] = mu * np.where(ok, np.maximum(t2 - t1, 0.0), 0.0) * np.linalg.norm(d, axis=-1)
    return out


def test_uniform_cylinder_reconstructs_its_attenuation():
    # off-centre cylinder, cone beam, 180 angles: interior mu within 1.5 %;
    # outside it (inside the 32 mm field of view) a zero mean, with streaks of
    # view sampling below 12 % of mu; the mirrored position empty
    g = synth.Geometry(sid=500.0, sdd=750.0, nu=160, nv=16, du=0.6, dv=0.6, n_angles=180)
    mu, R, x0, y0 = 0.02, 18.0, 12.0, -7.0
    proj = _cylinder_projections(g, mu, R, x0, y0, 40.0)
    grid = synth.Grid(nx=64, ny=64, nz=3, dx=1.0, dy=1.0, dz=1.0)
    vol = fdk.fdk(proj, g, grid)
    x, y, z = fdk.voxel_centres(grid)
    X, Yy = np.meshgrid(x, y, indexing="xy")
    r = np.hypot(X - x0, Yy - y0)
    mid = vol[1]
    fov = np.hypot(X, Yy) < 28.0
    inside = mid[r < R - 3.0]
    outside = mid[(r > R + 3.0) & fov]
    assert abs(inside.mean() / mu - 1.0) < 0.01, inside.mean() / mu
    assert np.abs(inside / mu - 1.0).max() < 0.015
    assert abs(outside.mean()) < 0.01 * mu and np.abs(outside).max() < 0.12 * mu
    rm = np.hypot(X + x0, Yy + y0)          # mirrored centre
    assert np.abs(mid[(rm < 5.0) & (r > R + 3.0)]).mean() < 0.03 * mu


def test_oracle_projector_round_trip(orc):
    # monoenergetic projections of a voxelised water cylinder by the projector
    # oracle (line integrals mu . L) reconstruct to mu in the interior
    h = 0.5
    labels = synth.cylinder_phantom(96, 96, 8, h, h, 20.0, [(6.0, 0.0, 4.0, 2)])
    ph = synth.Phantom(dx=h, dy=h, dz=h, labels=labels)
    g = synth.Geometry(sid=600.0, sdd=900.0, nu=128, nv=8, du=0.6, dv=0.6, n_angles=120)
    mus = np.array([0.0, 0.02, 0.035])
    L = orc.pathlengths(g, ph, 3, list(range(g.n_angles)))
    proj = L @ mus
    grid = synth.Grid(nx=48, ny=48, nz=1, dx=1.0, dy=1.0, dz=0.5, cz=0.25)
    vol = fdk.fdk(proj, g, grid)[0]
    x, y, _ = fdk.voxel_centres(grid)
    X, Yy = np.meshgrid(x, y, indexing="xy")
    water = (np.hypot(X, Yy) < 17.0) & (np.hypot(X - 6.0, Yy) > 6.5)
    insert = np.hypot(X - 6.0, Yy) < 2.0
    assert abs(vol[water].mean() / 0.02 - 1.0) < 0.015
    assert abs(vol[insert].mean() / 0.035 - 1.0) < 0.03


def test_short_source_distance_fan():
    # a wide fan (source 120 mm from the axis, object out to 40 mm): the cosine
    # weight, the D^2/U^2 weight and the side of the source each change the
    # mid-plane result by several per cent if wrong; FDK is exact there
    g = synth.Geometry(sid=120.0, sdd=240.0, nu=400, nv=4, du=0.5, dv=0.5, n_angles=360)
    mu, R, x0, y0 = 0.03, 14.0, 24.0, 10.0
    proj = _cylinder_projections(g, mu, R, x0, y0, 60.0)
    grid = synth.Grid(nx=96, ny=96, nz=1, dx=1.0, dy=1.0, dz=0.5)
    mid = fdk.fdk(proj, g, grid)[0]
    x, y, _ = fdk.voxel_centres(grid)
    X, Yy = np.meshgrid(x, y, indexing="xy")
    r = np.hypot(X - x0, Yy - y0)
    inside = mid[r < R - 2.5]
    assert abs(inside.mean() / mu - 1.0) < 0.01, inside.mean() / mu
    assert np.abs(inside / mu - 1.0).max() < 0.03
    outside = mid[(r > R + 2.5) & (np.hypot(X, Yy) < 45.0)]
    assert abs(outside.mean()) < 0.01 * mu


def test_axial_position():
    # a short cylinder above the mid-plane (2 < z < 8 mm) appears there and not
    # below it: pins the sign and scale of the axial detector coordinate
    g = synth.Geometry(sid=500.0, sdd=750.0, nu=128, nv=48, du=0.6, dv=0.6, n_angles=120, off_v=0.3)
    mu, R = 0.02, 15.0
    proj = _cylinder_projections(g, mu, R, 0.0, 0.0, 3.0, z0=5.0)
    grid = synth.Grid(nx=40, ny=40, nz=4, dx=1.0, dy=1.0, dz=1.0, cz=0.0)
    x, y, z = fdk.voxel_centres(grid)
    pts = np.array([[xx, yy, zz] for zz in (-5.0, 5.0) for yy in (-4.0, 0.0, 4.0) for xx in (-4.0, 0.0, 4.0)])
    vals = fdk.backproject(fdk.filter_projections(proj, g), g, pts).reshape(2, -1)
    assert np.abs(vals[0]).max() < 0.03 * mu
    assert np.abs(vals[1] / mu - 1.0).max() < 0.03


def test_backprojection_geometry_exact():
    # a single unit sample of the filtered projections at pixel (iv, iu) of
    # angle a reaches exactly the points on the ray from the source to that
    # pixel's centre, with weight (1/2)(2 pi / A) D^2 / U^2
    g = synth.Geometry(sid=300.0, sdd=520.0, nu=33, nv=21, du=0.7, dv=0.9, n_angles=10,
                       off_u=2.1, off_v=-3.3)
    a, iv, iu = 3, 5, 27
    filt = np.zeros((g.n_angles, g.nv, g.nu))
    filt[a, iv, iu] = 1.0
    b = g.angle_values()[a]
    cb, sb = math.cos(b), math.sin(b)
    src = np.array([g.sid * cb, g.sid * sb, 0.0])
    ctr = -(g.sdd - g.sid) * np.array([cb, sb, 0.0])
    pix = (ctr + ((iu - (g.nu - 1) / 2) * g.du + g.off_u) * np.array([-sb, cb, 0.0])
           + ((iv - (g.nv - 1) / 2) * g.dv + g.off_v) * np.array([0.0, 0.0, 1.0]))
    lam = np.array([0.35, 0.5, 0.62])
    pts = src[None] + lam[:, None] * (pix - src)[None]
    got = fdk.backproject(filt, g, pts)
    U = g.sid - (pts[:, 0] * cb + pts[:, 1] * sb)
    want = 0.5 * (2 * math.pi / g.n_angles) * g.sid ** 2 / U ** 2
    np.testing.assert_allclose(got, want, rtol=1e-9)
    # half a pixel away along u the bilinear weight is 1/2
    off = pts[1] + 0.5 * g.du * (U[1] / g.sdd) * np.array([-sb, cb, 0.0])
    np.testing.assert_allclose(fdk.backproject(filt, g, off[None]), 0.5 * want[1:2], rtol=1e-9)
