"""Pins of the dose oracle (oracle/dose.py), Sec. II.H, Eqs. 6-7.

Expected values: a hand-worked two-ray example; the uniform water cylinder,
whose chords have a closed form (2 sqrt(r^2 - d^2) in the plane, clipped by
the end faces); the opaque and thin limits; linearity in phi.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dose as od


def test_hand_worked_example():
    # two rays, two energies, one material; mu = (ln 2, ln 4) per mm
    # ray 0: L = 1 mm -> 1 - e^-P = (1/2, 3/4); ray 1: L = 0 -> (0, 0)
    # E = (10, 20), r = (0.5, 0.25): D0 = E r (sum over rays) / (2 * M), M = 5
    #   D0[0] = 10 * 0.5 * 0.5 / 10 = 0.25;  D0[1] = 20 * 0.25 * 0.75 / 10 = 0.375
    # phi = (0.4, 0.6): Dp = 0.1 + 0.225 = 0.325
    L = np.array([[1.0], [0.0]])
    mu = np.array([[math.log(2.0), math.log(4.0)]])
    D0, Dp = od.dose_per_particle(L, mu, [10.0, 20.0], [0.5, 0.25], [0.4, 0.6], 5.0)
    np.testing.assert_allclose(D0, [0.25, 0.375], rtol=1e-15)
    assert abs(Dp - 0.325) < 1e-15


def _cylinder_chords(geometry, R, half_h, angles):
    """Closed-form chord of every source-to-pixel ray through the cylinder
    x^2 + y^2 <= R^2, |z| <= half_h."""
    out = []
    for a in angles:
        t = geometry.angle_values()[a]
        c, s = math.cos(t), math.sin(t)
        src = np.array([geometry.sid * c, geometry.sid * s, 0.0])
        back = geometry.sdd - geometry.sid
        ctr = np.array([-back * c, -back * s, 0.0])
        eu, ev = np.array([-s, c, 0.0]), np.array([0.0, 0.0, 1.0])
        for iv in range(geometry.nv):
            for iu in range(geometry.nu):
                pix = (ctr + ((iu - (geometry.nu - 1) / 2) * geometry.du) * eu
                       + ((iv - (geometry.nv - 1) / 2) * geometry.dv) * ev)
                d = pix - src
                # x^2 + y^2 = R^2 along src + t d
                A = d[0] ** 2 + d[1] ** 2
                B = 2 * (src[0] * d[0] + src[1] * d[1])
                Cc = src[0] ** 2 + src[1] ** 2 - R * R
                disc = B * B - 4 * A * Cc
                if disc <= 0:
                    out.append(0.0)
                    continue
                t1, t2 = (-B - math.sqrt(disc)) / (2 * A), (-B + math.sqrt(disc)) / (2 * A)
                if d[2] != 0.0:
                    z1, z2 = sorted(((-half_h - src[2]) / d[2], (half_h - src[2]) / d[2]))
                    t1, t2 = max(t1, z1), min(t2, z2)
                t1, t2 = max(t1, 0.0), min(t2, 1.0)
                out.append(max(t2 - t1, 0.0) * float(np.linalg.norm(d)))
    return np.array(out)


def test_uniform_water_cylinder_closed_form(orc):
    # voxelised water cylinder (r = 20 mm, 0.25 mm voxels) against the exact chords
    R, h, nz = 20.0, 0.25, 24
    n = 176
    labels = synth.cylinder_phantom(n, n, nz, h, h, R, [])
    ph = synth.Phantom(dx=h, dy=h, dz=h, labels=labels)
    g = synth.Geometry(sid=1000.0, sdd=1500.0, nu=72, nv=12, du=1.0, dv=0.75, n_angles=8)
    angles = [0, 3, 5]
    L = orc.pathlengths(g, ph, 2, angles)
    x_exact = _cylinder_chords(g, R, nz * h / 2, angles)
    E = np.array([0.03, 0.06, 1.0])
    mu_w = np.array([0.037, 0.021, 0.0071])        # per mm
    r = np.array([0.8, 0.15, 0.45])
    phi = np.array([0.2, 0.5, 0.3])
    mu = np.stack([np.zeros(3), mu_w])
    D0, Dp = od.dose_per_particle(L, mu, E, r, phi, 1.0)
    ref = E * r * (-np.expm1(-np.outer(x_exact, mu_w))).sum(axis=0) / x_exact.size
    # staircase boundary: a chord is off by up to ~h at the rim, and the
    # errors of the two crossings mostly cancel in the mean (measured 5e-4)
    np.testing.assert_allclose(D0, ref, rtol=3e-3)
    assert abs(Dp - float((phi * ref).sum())) < 3e-3 * Dp
    # the detector is wider than the cylinder: some rays miss and still count in N_i
    assert 0.3 * x_exact.size < np.count_nonzero(x_exact) < x_exact.size


def test_opaque_and_thin_limits():
    rng = np.random.default_rng(3)
    L = rng.uniform(0.0, 30.0, (500, 2))
    L[:80] = 0.0                                    # rays that miss
    E, r, phi = np.array([2.0]), np.array([0.7]), np.array([1.0])
    # opaque: every hit photon deposits E r
    D0, _ = od.dose_per_particle(L, np.array([[1e6], [1e6]]), E, r, phi, 3.0)
    np.testing.assert_allclose(D0, [2.0 * 0.7 * 420 / (500 * 3.0)], rtol=1e-15)
    # thin: 1 - e^-P ~ P, so D0 ~ E r sum_i P_i / (N M), relative error ~ P / 2
    mu = np.array([[1e-9], [2e-9]])
    D0, _ = od.dose_per_particle(L, mu, E, r, phi, 3.0)
    lin = 2.0 * 0.7 * (L @ mu[:, 0]).sum() / (500 * 3.0)
    assert abs(D0[0] / lin - 1.0) < 1e-7


def test_linear_in_phi_and_mass():
    rng = np.random.default_rng(4)
    L = rng.uniform(0.0, 10.0, (64, 3))
    mu = rng.uniform(0.0, 0.1, (3, 5))
    E, r = rng.uniform(0.02, 6.0, 5), rng.uniform(0.1, 0.9, 5)
    p1, p2 = rng.random(5), rng.random(5)
    D0a, Da = od.dose_per_particle(L, mu, E, r, p1, 2.0)
    D0b, Db = od.dose_per_particle(L, mu, E, r, p2, 2.0)
    D0c, Dc = od.dose_per_particle(L, mu, E, r, 2 * p1 + p2, 4.0)
    np.testing.assert_array_equal(D0a, D0b)
    np.testing.assert_allclose(D0c, D0a / 2, rtol=1e-15)
    assert abs(Dc - (2 * Da + Db) / 2) < 1e-14 * abs(Dc)
