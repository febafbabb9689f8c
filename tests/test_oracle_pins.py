"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
a closed form, a construction whose answer is known, an independent
brute-force sampler, a library routine (SciPy / NumPy convolution), an
invariant, or the hand-worked example under ``tests/golden/``.

Passages: Sec. II.F (projection = line integral of attenuation along the
ray; Eq. 3 spectral sum with scatter added to the primary profiles),
Sec. II.C (labelled phantom: mu(E, x) = mu_label(x)(E)), Sec. II.G (each
group's profile convolved with its optical spread kernel, then summed).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.signal

from synth import Geometry, Phantom

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def vol(labels, h=(1.0, 1.0, 1.0), c=(0.0, 0.0, 0.0)):
    return Phantom(dx=h[0], dy=h[1], dz=h[2], labels=np.ascontiguousarray(labels, dtype=np.int8),
                   cx=c[0], cy=c[1], cz=c[2])


# --------------------------------------------------------------- geometry

def test_geometry_conventions(orc):
    g = Geometry(sid=1000.0, sdd=1500.0, nu=5, nv=3, du=2.0, dv=3.0, n_angles=4)
    s, p = orc.ray_endpoints(g, 0, 1, 2)             # centre pixel, theta = 0
    np.testing.assert_allclose(s, [1000.0, 0.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(p, [-500.0, 0.0, 0.0], atol=1e-12)
    assert abs(np.linalg.norm(p - s) - 1500.0) < 1e-9
    # one pixel along u moves by du along (-sin t, cos t, 0); along v by dv along +z
    _, pu = orc.ray_endpoints(g, 0, 1, 3)
    _, pv = orc.ray_endpoints(g, 0, 2, 2)
    np.testing.assert_allclose(pu - p, [0.0, 2.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(pv - p, [0.0, 0.0, 3.0], atol=1e-12)
    # a = 1 of 4 is theta = pi/2: source on +y, u axis along -x
    s1, p1 = orc.ray_endpoints(g, 1, 1, 3)
    np.testing.assert_allclose(s1, [0.0, 1000.0, 0.0], atol=1e-9)
    np.testing.assert_allclose(p1, [-2.0, -500.0, 0.0], atol=1e-9)
    # detector offsets shift the pixel centre
    g2 = Geometry(sid=1000.0, sdd=1500.0, nu=5, nv=3, du=2.0, dv=3.0, n_angles=4, off_u=0.5, off_v=-0.25)
    _, po = orc.ray_endpoints(g2, 0, 1, 2)
    np.testing.assert_allclose(po, [-500.0, 0.5, -0.25], atol=1e-12)
    # explicit angles override 2 pi a / A
    g3 = Geometry(sid=1000.0, sdd=1500.0, nu=5, nv=3, du=2.0, dv=3.0, n_angles=1,
                  angles=np.array([math.pi]))
    s3, _ = orc.ray_endpoints(g3, 0, 1, 2)
    np.testing.assert_allclose(s3, [-1000.0, 0.0, 0.0], atol=1e-9)


# ------------------------------------------------------------ path lengths

def test_single_voxel_pins_axis_order_and_sizes(orc):
    """One labelled voxel in a non-cubic, anisotropic grid: only the ray through
    its world position (x0 + (i+1/2) h per axis) sees it, for exactly h."""
    lab = np.zeros((3, 4, 5), dtype=np.int8)       # nz, ny, nx
    lab[2, 1, 3] = 1                                # iz=2, iy=1, ix=3
    ph = vol(lab, h=(1.0, 2.0, 0.5))
    # x0 = -2.5, y0 = -4, z0 = -0.75 -> centre (1.0, -1.0, 0.5)
    Lx = orc.siddon([-10, -1.0, 0.5], [10, -1.0, 0.5], ph, 2)
    Ly = orc.siddon([1.0, -10, 0.5], [1.0, 10, 0.5], ph, 2)
    Lz = orc.siddon([1.0, -1.0, -10], [1.0, -1.0, 10], ph, 2)
    np.testing.assert_allclose(Lx, [4.0, 1.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Ly, [6.0, 2.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Lz, [1.0, 0.5], rtol=0, atol=1e-12)
    # a neighbouring line never sees it
    assert orc.siddon([-10, 1.0, 0.5], [10, 1.0, 0.5], ph, 2)[1] == 0.0
    # volume centre offset moves the grid
    ph2 = vol(lab, h=(1.0, 2.0, 0.5), c=(10.0, 0.0, 0.0))
    np.testing.assert_allclose(orc.siddon([0, -1.0, 0.5], [20, -1.0, 0.5], ph2, 2), [4.0, 1.0], atol=1e-12)


def _box_surface_point(rng, lo, hi, face):
    p = rng.uniform(lo, hi)
    ax, side = divmod(face, 2)
    p[ax] = lo[ax] if side == 0 else hi[ax]
    return p


@pytest.mark.parametrize("seed", range(4))
def test_total_length_is_chord(orc, seed):
    """Entry and exit points are drawn on two faces of the grid, so the chord
    is |exit - entry| by construction; sum_m L_m equals it for any labels."""
    rng = np.random.default_rng(seed)
    n = (7, 5, 6)
    h = (0.7, 1.3, 0.9)
    lab = rng.integers(0, 4, size=(n[2], n[1], n[0]))
    ph = vol(lab, h=h)
    hi = np.array([n[0] * h[0], n[1] * h[1], n[2] * h[2]]) / 2
    lo = -hi
    for _ in range(50):
        f0, f1 = rng.choice(6, size=2, replace=False)
        a = _box_surface_point(rng, lo, hi, f0)
        b = _box_surface_point(rng, lo, hi, f1)
        src = a - rng.uniform(0.1, 3.0) * (b - a)
        dst = b + rng.uniform(0.1, 3.0) * (b - a)
        L = orc.siddon(src, dst, ph, 4)
        chord = np.linalg.norm(b - a)
        assert abs(L.sum() - chord) <= 1e-12 * max(1.0, chord)
        # a segment that stops inside the grid sees only the part inside
        mid = a + 0.5 * (b - a)
        Lh = orc.siddon(src, mid, ph, 4)
        assert abs(Lh.sum() - 0.5 * chord) <= 1e-12 * max(1.0, chord)
    # rays that miss the grid see nothing
    assert orc.siddon([20, 20, 0], [30, -20, 0], ph, 4).sum() == 0.0


def test_lattice_rays(orc):
    rng = np.random.default_rng(7)
    N = 6
    h = 0.8
    lab = rng.integers(0, 5, size=(N, N, N))
    ph = vol(lab, h=(h, h, h))
    c = lambda i: -N * h / 2 + (i + 0.5) * h
    for iz in range(N):
        for iy in range(N):
            L = orc.siddon([-50, c(iy), c(iz)], [50, c(iy), c(iz)], ph, 5)
            want = np.bincount(lab[iz, iy, :], minlength=5) * h
            np.testing.assert_allclose(L, want, atol=1e-12)
            Ly = orc.siddon([c(iy), 50, c(iz)], [c(iy), -50, c(iz)], ph, 5)   # negative direction
            np.testing.assert_allclose(Ly, np.bincount(lab[iz, :, iy], minlength=5) * h, atol=1e-12)
    # in-plane diagonal through voxel centres (i, i, k): h*sqrt(2) per voxel
    for iz in range(N):
        L = orc.siddon([c(-20), c(-20), c(iz)], [c(30), c(30), c(iz)], ph, 5)
        want = np.bincount([lab[iz, i, i] for i in range(N)], minlength=5) * h * math.sqrt(2)
        np.testing.assert_allclose(L, want, atol=1e-12)
    # space diagonal through voxel centres (i, i, i): h*sqrt(3) per voxel
    L = orc.siddon([c(-20)] * 3, [c(30)] * 3, ph, 5)
    want = np.bincount([lab[i, i, i] for i in range(N)], minlength=5) * h * math.sqrt(3)
    np.testing.assert_allclose(L, want, atol=1e-12)


def test_slab_and_monoenergetic_beer_lambert(orc):
    """A slab with faces on voxel planes: L = t |d| / |d_x| exactly; one bin of
    unit weight gives I0 exp(-mu t |d|/|d_x|)."""
    nx, ny, nz, h = 20, 8, 8, 0.5
    lab = np.zeros((nz, ny, nx), dtype=np.int8)
    lab[:, :, 6:13] = 2                               # t = 7 * 0.5 = 3.5 mm
    ph = vol(lab, h=(h, h, h))
    rng = np.random.default_rng(3)
    mu = np.array([[0.0], [0.0], [0.37]])
    for _ in range(20):
        src = np.array([-30.0, rng.uniform(-1, 1), rng.uniform(-1, 1)])
        dst = np.array([30.0, rng.uniform(-1, 1), rng.uniform(-1, 1)])
        d = dst - src
        L = orc.siddon(src, dst, ph, 3)
        want = 3.5 * np.linalg.norm(d) / abs(d[0])
        assert abs(L[2] - want) <= 1e-12 * want
        Y = orc.spectral(L[None, :], mu, [1.0], [1.0], [0], 1, i0=[1.7])
        assert abs(Y[0, 0] - 1.7 * math.exp(-0.37 * want)) <= 1e-14


@pytest.mark.parametrize("shape", ["cylinder", "sphere"])
def test_voxelised_body_converges_to_analytic_chord(orc, shape):
    """Centre-in voxelisation of a radius-r body: |L - 2 sqrt(r^2 - d^2)| <= 2 sqrt(3) h,
    and the mean error at least halves as h halves."""
    r = 10.0
    rng = np.random.default_rng(11)
    offs = rng.uniform(0.0, 0.9 * r, size=40)
    angs = rng.uniform(0, 2 * np.pi, size=40)
    errs = []
    for h in (1.0, 0.5, 0.25):
        n = int(round(2 * (r + 2) / h))
        ctr = -n * h / 2 + (np.arange(n) + 0.5) * h
        if shape == "cylinder":
            nz = 2
            body = (ctr[None, :] ** 2 + ctr[:, None] ** 2) <= r * r
            lab = np.broadcast_to(body, (nz, n, n)).astype(np.int8)
            ph = vol(lab, h=(h, h, h))
        else:
            body = (ctr[None, None, :] ** 2 + ctr[None, :, None] ** 2 + ctr[:, None, None] ** 2) <= r * r
            lab = body.astype(np.int8)
            ph = vol(lab, h=(h, h, h))
        e = []
        for d, t in zip(offs, angs):
            dirv = np.array([math.cos(t), math.sin(t), 0.0])
            perp = np.array([-math.sin(t), math.cos(t), 0.0])
            z = 0.3 * h if shape == "cylinder" else 0.0
            base = d * perp + np.array([0, 0, z])
            L = orc.siddon(base - 40 * dirv, base + 40 * dirv, ph, 2)
            chord = 2 * math.sqrt(r * r - d * d)
            assert abs(L[1] - chord) <= 2 * math.sqrt(3) * h
            e.append(abs(L[1] - chord))
        errs.append(np.mean(e))
    assert errs[1] <= 0.75 * errs[0] and errs[2] <= 0.75 * errs[1]


@pytest.mark.parametrize("seed", range(3))
def test_siddon_matches_brute_force(orc, seed):
    rng = np.random.default_rng(100 + seed)
    lab = rng.integers(0, 4, size=(4, 5, 6))
    ph = vol(lab, h=(1.1, 0.9, 1.3))
    for _ in range(6):
        src = rng.uniform(-6, 6, size=3)
        dst = rng.uniform(-6, 6, size=3)
        L = orc.siddon(src, dst, ph, 4)
        n_steps = 1_000_000
        Lb = orc.bruteforce(src, dst, ph, 4, n_steps)
        step = np.linalg.norm(dst - src) / n_steps
        assert np.all(np.abs(L - Lb) <= step * (6 + 5 + 4 + 3))


def test_rotation_symmetry(orc):
    """Rotating the phantom by +90 deg about z and the gantry by +90 deg gives the same L per pixel."""
    rng = np.random.default_rng(5)
    N, nz = 12, 3
    lab = rng.integers(0, 4, size=(nz, N, N)).astype(np.int8)
    # new(x', y') = old(y', -x')  ->  new[k][j'][i'] = old[k][N-1-i'][j']
    ip, jp = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    rot = lab[:, N - 1 - ip, jp]
    t = 0.4321
    g0 = Geometry(sid=200.0, sdd=300.0, nu=24, nv=5, du=0.9, dv=0.7, n_angles=1, angles=np.array([t]))
    g1 = Geometry(sid=200.0, sdd=300.0, nu=24, nv=5, du=0.9, dv=0.7, n_angles=1,
                  angles=np.array([t + np.pi / 2]))
    L0 = orc.pathlengths(g0, vol(lab, h=(0.6, 0.6, 0.6)), 4, [0])
    L1 = orc.pathlengths(g1, vol(rot, h=(0.6, 0.6, 0.6)), 4, [0])
    assert L0.sum() > 0
    np.testing.assert_allclose(L1, L0, rtol=1e-12, atol=1e-12)


def test_bad_label_is_reported(orc):
    lab = np.zeros((2, 2, 2), dtype=np.int8)
    lab[0, 0, 0] = 5
    with pytest.raises(ValueError):
        orc.siddon([-5, -0.5, -0.5], [5, -0.5, -0.5], vol(lab), 3)


# -------------------------------------------------------------- spectral

def test_spectral_worked_example(orc):
    """Hand-worked example (tests/golden/spectral_worked_example.json)."""
    with open(os.path.join(GOLDEN, "spectral_worked_example.json")) as f:
        ex = json.load(f)
    ln2, ln3 = math.log(2.0), math.log(3.0)
    mu = np.array([[ln2, 0.0, ln3], [0.0, ln2 / 2, ln3 / 2]])
    for case in ex["cases"]:
        Y = orc.spectral(np.array([ex["L"]]), mu, ex["phi"], ex["eta"], ex["group_of_bin"], 2,
                         i0=[case["I0"]], S=[case["S"]], s_bin=case["s_bin"])
        np.testing.assert_allclose(Y[:, 0], case["Y"], rtol=1e-14, atol=1e-15)


def test_spectral_identities(orc):
    rng = np.random.default_rng(9)
    n, M, E, G = 50, 5, 24, 3
    L = rng.uniform(0, 40, size=(n, M))
    mu = rng.uniform(0.0, 0.08, size=(M, E))
    phi = rng.uniform(0.1, 1.0, size=E)
    eta = rng.uniform(0.2, 1.0, size=E)
    grp = np.sort(rng.integers(0, G, size=E))
    S = rng.uniform(0, 0.2, size=n)
    i0 = rng.uniform(0.5, 2.0, size=n)
    sb = rng.uniform(0.5, 1.5, size=E)
    Y = orc.spectral(L, mu, phi, eta, grp, G, i0=i0, S=S, s_bin=sb)
    w = phi * eta
    W = np.array([w[grp == g].sum() for g in range(G)])
    Ws = np.array([(w * sb)[grp == g].sum() for g in range(G)])
    # L = 0: Y_g = I0 W_g + Ws_g S
    Y0 = orc.spectral(np.zeros((n, M)), mu, phi, eta, grp, G, i0=i0, S=S, s_bin=sb)
    np.testing.assert_allclose(Y0, W[:, None] * i0[None] + Ws[:, None] * S[None], rtol=1e-14)
    # linear in phi
    phi2 = rng.uniform(0.1, 1.0, size=E)
    Ya = orc.spectral(L, mu, phi + 2 * phi2, eta, grp, G, i0=i0, S=S, s_bin=sb)
    Yb = orc.spectral(L, mu, phi2, eta, grp, G, i0=i0, S=S, s_bin=sb)
    np.testing.assert_allclose(Ya, Y + 2 * Yb, rtol=1e-13)
    # splitting every bin into two halves changes nothing
    Y2 = orc.spectral(L, np.repeat(mu, 2, axis=1), np.repeat(phi / 2, 2), np.repeat(eta, 2),
                      np.repeat(grp, 2), G, i0=i0, S=S, s_bin=np.repeat(sb, 2))
    np.testing.assert_allclose(Y2, Y, rtol=1e-13)
    # permuting materials (columns of L with rows of mu) changes nothing
    perm = rng.permutation(M)
    Yp = orc.spectral(L[:, perm], mu[perm], phi, eta, grp, G, i0=i0, S=S, s_bin=sb)
    np.testing.assert_allclose(Yp, Y, rtol=1e-13)
    # more material never brightens a pixel; the total equals the ungrouped sum
    Lm = L.copy()
    Lm[:, 2] += 1.0
    assert np.all(orc.spectral(Lm, mu, phi, eta, grp, G, i0=i0) <= orc.spectral(L, mu, phi, eta, grp, G, i0=i0))
    Y1 = orc.spectral(L, mu, phi, eta, np.zeros(E, np.int32), 1, i0=i0, S=S, s_bin=sb)
    np.testing.assert_allclose(Y1[0], Y.sum(axis=0), rtol=1e-13)


# ------------------------------------------------------------------- psf

def test_psf_against_library_convolution(orc):
    rng = np.random.default_rng(12)
    A, G, nv, nu, k = 2, 3, 19, 33, 7
    Y = rng.uniform(0, 1, size=(A, G, nv, nu))
    K = rng.uniform(0, 1, size=(G, k, k))
    out = orc.psf(Y, K)
    for a in range(A):
        want = sum(scipy.signal.convolve2d(Y[a, g], K[g], mode="same", boundary="fill") for g in range(G))
        np.testing.assert_allclose(out[a], want, rtol=1e-12)
        # and via the FFT: full linear convolution, cropped to the centre
        c = (k - 1) // 2
        full = sum(np.real(np.fft.ifft2(np.fft.fft2(Y[a, g], s=(nv + k - 1, nu + k - 1)) *
                                        np.fft.fft2(K[g], s=(nv + k - 1, nu + k - 1)))) for g in range(G))
        np.testing.assert_allclose(out[a], full[c:c + nv, c:c + nu], rtol=1e-9, atol=1e-12)


def test_psf_delta_shift_pins_flip(orc):
    rng = np.random.default_rng(13)
    nv, nu, k = 9, 11, 5
    Y = rng.uniform(0, 1, size=(1, 1, nv, nu))
    c = (k - 1) // 2
    K = np.zeros((1, k, k))
    K[0, c, c] = 1.0
    np.testing.assert_array_equal(orc.psf(Y, K), Y[:, 0])
    # K[p][q] = 1 moves the image by (p - c, q - c): out[v][u] = Y[v - (p-c)][u - (q-c)]
    p, q = 4, 1
    K = np.zeros((1, k, k))
    K[0, p, q] = 1.0
    out = orc.psf(Y, K)[0]
    want = np.zeros((nv, nu))
    sv, su = p - c, q - c
    for v in range(nv):
        for u in range(nu):
            if 0 <= v - sv < nv and 0 <= u - su < nu:
                want[v, u] = Y[0, 0, v - sv, u - su]
    np.testing.assert_array_equal(out, want)


def test_psf_separable_and_mass(orc):
    rng = np.random.default_rng(14)
    nv, nu, k = 30, 40, 9
    gv = rng.uniform(0, 1, size=k)
    gu = rng.uniform(0, 1, size=k)
    Y = np.zeros((1, 1, nv, nu))
    Y[0, 0, 8:22, 8:32] = rng.uniform(0, 1, size=(14, 24))   # zero border wider than the kernel
    out = orc.psf(Y, np.outer(gv, gu)[None])[0]
    rows = np.array([np.convolve(r, gu, mode="same") for r in Y[0, 0]])
    both = np.array([np.convolve(col, gv, mode="same") for col in rows.T]).T
    np.testing.assert_allclose(out, both, rtol=1e-12, atol=1e-15)
    assert abs(out.sum() - Y.sum() * gv.sum() * gu.sum()) <= 1e-10 * out.sum()


# ------------------------------------------------------- whole projector

def test_project_uniform_slab_end_to_end(orc):
    """Full pipeline on a uniform slab, one bin, no scatter/psf: closed-form Beer-Lambert per pixel."""
    from synth import Config, Spectral
    nx, ny, nz, h = 40, 40, 6, 0.5
    lab = np.zeros((nz, ny, nx), dtype=np.int8)
    lab[:, :, 14:26] = 1                                     # slab |x| < 3 mm
    g = Geometry(sid=100.0, sdd=150.0, nu=9, nv=5, du=1.0, dv=1.0, n_angles=1, angles=np.array([0.0]))
    sp = Spectral(energies=np.array([60.0]), mu=np.array([[0.0], [0.2]], dtype=np.float32),
                  phi=np.array([1.0], np.float32), eta=np.array([1.0], np.float32), n_groups=1,
                  group_of_bin=np.array([0], np.int32))
    cfg = Config("slab", g, vol(lab, h=(h, h, h)), sp)
    out = orc.project(cfg, [0])
    for iv in range(5):
        for iu in range(9):
            s, p = orc.ray_endpoints(g, 0, iv, iu)
            d = p - s
            Lw = 6.0 * np.linalg.norm(d) / abs(d[0])
            assert abs(out[0, iv, iu] - math.exp(-np.float32(0.2) * Lw)) <= 1e-14
