"""FP64 oracle of the FDK reconstruction (test infrastructure only).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the product library never does.

The paper reconstructs its projections with the default FDK algorithm of its
toolkit (Sec. II.G; Feldkamp, Davis and Kress, J. Opt. Soc. Am. A 1 (1984)
612).  Written here from that algorithm, in the geometry of this library:

* source at D (cos b, sin b, 0) with D = SID; the detector at distance
  SDD from the source; its u axis (-sin b, cos b, 0) and v axis z;
* the projections are rescaled to a virtual detector through the rotation
  axis: a = u_det D / SDD, c = v_det D / SDD (pixel pitch tau = du D / SDD);
* cosine weight D / sqrt(D^2 + a^2 + c^2);
* ramp filter along each detector row: the band-limited (Ram-Lak) kernel in
  the spatial domain, h(0) = 1 / (4 tau^2), h(n tau) = 0 for even n != 0,
  -1 / (n^2 pi^2 tau^2) for odd n (Kak and Slaney, "Principles of
  Computerized Tomographic Imaging", Ch. 3), as a full linear convolution
  with zeros beyond the detector, times tau;
* back-projection: a voxel at (x, y, z) with s = x cos b + y sin b,
  t = -x sin b + y cos b and U = D - s meets the virtual detector at
  a = D t / U, c = D z / U; the filtered row is sampled there by bilinear
  interpolation (zero outside the detector) and weighted by D^2 / U^2;
* f = (1/2) (2 pi / A) sum over the A angles (a full, evenly spaced scan
  measures every line twice).
The result is the attenuation coefficient in the unit of 1 / length of the
geometry (mm^-1).
"""
from __future__ import annotations

import math

import numpy as np


def ramp_kernel(n: int, tau: float) -> np.ndarray:
    """tau h(k tau) for k = -(n - 1) .. n - 1 (Ram-Lak, spatial domain)."""
    k = np.arange(-(n - 1), n)
    h = np.zeros(k.size)
    h[k == 0] = 1.0 / (4.0 * tau * tau)
    odd = (k % 2) != 0
    h[odd] = -1.0 / (k[odd].astype(np.float64) ** 2 * math.pi ** 2 * tau * tau)
    return h * tau


def virtual_coordinates(geometry):
    """(a[nu], c[nv]): pixel centres scaled to the virtual detector at the axis."""
    g = geometry
    mag = g.sid / g.sdd
    a = ((np.arange(g.nu) - (g.nu - 1) / 2.0) * g.du + g.off_u) * mag
    c = ((np.arange(g.nv) - (g.nv - 1) / 2.0) * g.dv + g.off_v) * mag
    return a, c


def filter_projections(proj, geometry) -> np.ndarray:
    """Cosine-weighted, ramp-filtered projections [A][nv][nu] (FP64)."""
    g = geometry
    proj = np.asarray(proj, np.float64)
    a, c = virtual_coordinates(g)
    D = g.sid
    w = D / np.sqrt(D * D + a[None, :] ** 2 + c[:, None] ** 2)
    q = proj * w[None]
    h = ramp_kernel(g.nu, g.du * g.sid / g.sdd)
    out = np.empty_like(q)
    for ai in range(q.shape[0]):
        for iv in range(g.nv):
            out[ai, iv] = np.convolve(q[ai, iv], h, mode="full")[g.nu - 1:2 * g.nu - 1]
    return out


def voxel_centres(grid):
    """Centre coordinates (x[nx], y[ny], z[nz]) of a grid (origin-centred boxes)."""
    x = grid.cx - grid.nx * grid.dx / 2.0 + (np.arange(grid.nx) + 0.5) * grid.dx
    y = grid.cy - grid.ny * grid.dy / 2.0 + (np.arange(grid.ny) + 0.5) * grid.dy
    z = grid.cz - grid.nz * grid.dz / 2.0 + (np.arange(grid.nz) + 0.5) * grid.dz
    return x, y, z


def _bilinear(row_img, iv_f, iu_f):
    """Bilinear sample of row_img [nv][nu] at fractional indices, zero outside."""
    nv, nu = row_img.shape
    i0 = np.floor(iu_f).astype(np.int64)
    j0 = np.floor(iv_f).astype(np.int64)
    fu = iu_f - i0
    fv = iv_f - j0
    out = np.zeros(np.broadcast(iu_f, iv_f).shape)
    for dj, wv in ((0, 1.0 - fv), (1, fv)):
        for di, wu in ((0, 1.0 - fu), (1, fu)):
            jj, ii = j0 + dj, i0 + di
            ok = (jj >= 0) & (jj < nv) & (ii >= 0) & (ii < nu)
            val = np.where(ok, row_img[np.clip(jj, 0, nv - 1), np.clip(ii, 0, nu - 1)], 0.0)
            out += wv * wu * val
    return out


def backproject(filtered, geometry, points) -> np.ndarray:
    """FDK back-projection of filtered projections at points [n][3] (x, y, z)."""
    g = geometry
    filtered = np.asarray(filtered, np.float64)
    P = np.asarray(points, np.float64).reshape(-1, 3)
    D = g.sid
    scale = g.sdd / g.sid
    f = np.zeros(P.shape[0])
    for ai, b in enumerate(g.angle_values()):
        cb, sb = math.cos(b), math.sin(b)
        s = P[:, 0] * cb + P[:, 1] * sb
        t = -P[:, 0] * sb + P[:, 1] * cb
        U = D - s
        a = D * t / U
        c = D * P[:, 2] / U
        iu_f = (a * scale - g.off_u) / g.du + (g.nu - 1) / 2.0
        iv_f = (c * scale - g.off_v) / g.dv + (g.nv - 1) / 2.0
        f += (D * D / (U * U)) * _bilinear(filtered[ai], iv_f, iu_f)
    return f * (0.5 * 2.0 * math.pi / g.n_angles)


def grid_points(grid, index=None) -> np.ndarray:
    """Centres of all voxels [nz][ny][nx] as [n][3], or of the voxels (iz, iy, ix) listed."""
    x, y, z = voxel_centres(grid)
    if index is None:
        Z, Yy, X = np.meshgrid(z, y, x, indexing="ij")
        return np.stack([X.ravel(), Yy.ravel(), Z.ravel()], axis=1)
    idx = np.asarray(index).reshape(-1, 3)
    return np.stack([x[idx[:, 2]], y[idx[:, 1]], z[idx[:, 0]]], axis=1)


def fdk(proj, geometry, grid) -> np.ndarray:
    """Reconstruction [nz][ny][nx] (FP64) from projections [A][nv][nu]."""
    filt = filter_projections(proj, geometry)
    vol = backproject(filt, geometry, grid_points(grid))
    return vol.reshape(grid.nz, grid.ny, grid.nx)
