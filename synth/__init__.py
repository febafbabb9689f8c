"""Seeded synthetic inputs for the polyenergetic cone-beam projector.

This module builds the arrays that stand in for the paper's Monte Carlo and
database inputs (Sec. II.A spectra, Sec. II.B detector response and optical
spread functions, Sec. II.C labelled phantoms and material attenuation tables,
Sec. II.E scatter).  None of those data sets ship with the paper, so every
array here is generated from a fixed seed with the shapes, sizes and value
ranges of the paper's workloads.

It holds none of the projector's arithmetic: no ray tracing, no attenuation,
no spectral weighting, no convolution.  Both the FP64 oracle and the HIP path
consume exactly the same bytes from here.

Units: millimetres for lengths, mm^-1 for attenuation coefficients, keV or MeV
for photon energies (stated per configuration), pixels for scatter and PSF
shapes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import json
import os

import numpy as np

__all__ = [
    "Geometry", "Phantom", "Spectral", "Scatter", "Psf", "Config",
    "make_config", "config_seed", "random_phantom", "material_tables",
    "kramers_spectrum", "detector_response", "gaussian_psfs", "refine_spectral",
]

SEED_BASE = 4736 * 10


def config_seed(n: int) -> int:
    """Seed of configuration ``n`` (NumPy PCG64)."""
    return SEED_BASE + int(n)


# ---------------------------------------------------------------- containers

@dataclass
class Geometry:
    """Circular cone-beam geometry (z is the rotation axis, isocentre at 0).

    ``angles`` is None for the evenly spaced full rotation theta_a = 2*pi*a/A.
    """
    sid: float
    sdd: float
    nu: int
    nv: int
    du: float
    dv: float
    n_angles: int
    off_u: float = 0.0
    off_v: float = 0.0
    angles: Optional[np.ndarray] = None  # float64 [A] radians, or None

    def angle_values(self) -> np.ndarray:
        if self.angles is not None:
            return np.asarray(self.angles, dtype=np.float64)
        return 2.0 * np.pi * np.arange(self.n_angles, dtype=np.float64) / self.n_angles


@dataclass
class Phantom:
    """Labelled voxel phantom, ``labels[z][y][x]`` int8 with values 0..M-1."""
    dx: float
    dy: float
    dz: float
    labels: np.ndarray
    cx: float = 0.0
    cy: float = 0.0
    cz: float = 0.0

    @property
    def nz(self) -> int:
        return int(self.labels.shape[0])

    @property
    def ny(self) -> int:
        return int(self.labels.shape[1])

    @property
    def nx(self) -> int:
        return int(self.labels.shape[2])


@dataclass
class Grid:
    """Reconstruction grid: nx x ny x nz voxels of dx x dy x dz mm, centred at
    (cx, cy, cz); voxel (ix, iy, iz) has its centre at
    c - n h / 2 + (i + 1/2) h per axis, as for a Phantom."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    cx: float = 0.0
    cy: float = 0.0
    cz: float = 0.0


@dataclass
class Spectral:
    """Per-material attenuation, source spectrum and detector response.

    ``mu[m][e]`` in mm^-1, ``phi[e]`` normalised to sum 1, ``eta[e]`` in (0, 1],
    ``group_of_bin[e]`` non-decreasing in 0..G-1, ``flood`` None (=1) or [nv][nu].
    """
    energies: np.ndarray
    mu: np.ndarray
    phi: np.ndarray
    eta: np.ndarray
    n_groups: int
    group_of_bin: np.ndarray
    flood: Optional[np.ndarray] = None
    energy_unit: str = "keV"
    material_names: Sequence[str] = ()

    @property
    def n_mat(self) -> int:
        return int(self.mu.shape[0])

    @property
    def n_energy(self) -> int:
        return int(self.mu.shape[1])


@dataclass
class Scatter:
    """Per-angle scatter maps: one anisotropic Gaussian blob per angle.

    The maps are produced on demand by :meth:`maps` so that large
    configurations need not hold all angles in memory at once.
    """
    nu: int
    nv: int
    amp: np.ndarray      # [A]
    cu: np.ndarray       # [A] pixel-index centre along u
    cv: np.ndarray       # [A]
    su: np.ndarray       # [A] sigma along u, pixels
    sv: np.ndarray       # [A]
    s_bin: Optional[np.ndarray] = None  # [E] float32 or None (=1)

    def maps(self, angle_index: Sequence[int] | np.ndarray | None = None) -> np.ndarray:
        if angle_index is None:
            angle_index = np.arange(self.amp.shape[0])
        idx = np.asarray(angle_index, dtype=np.int64).reshape(-1)
        u = np.arange(self.nu, dtype=np.float64)
        v = np.arange(self.nv, dtype=np.float64)
        out = np.empty((idx.size, self.nv, self.nu), dtype=np.float32)
        for k, a in enumerate(idx):
            gu = np.exp(-0.5 * ((u - self.cu[a]) / self.su[a]) ** 2)
            gv = np.exp(-0.5 * ((v - self.cv[a]) / self.sv[a]) ** 2)
            out[k] = (self.amp[a] * gv[:, None] * gu[None, :]).astype(np.float32)
        return out


@dataclass
class Psf:
    """Per energy-group optical spread kernels ``kernels[g][k][k]`` (k odd)."""
    kernels: np.ndarray

    @property
    def k(self) -> int:
        return int(self.kernels.shape[1])


@dataclass
class Config:
    name: str
    geometry: Geometry
    phantom: Phantom
    spectral: Spectral
    scatter: Optional[Scatter] = None
    psf: Optional[Psf] = None
    mode: str = "plain"
    notes: dict = field(default_factory=dict)

    @property
    def rays(self) -> int:
        g = self.geometry
        return g.n_angles * g.nu * g.nv

    @property
    def ray_energy(self) -> int:
        return self.rays * self.spectral.n_energy


# ------------------------------------------------------------ spectral inputs

# Tissue-like parameter sets, made up for this synthetic stand-in (no
# database values): (relative density, photoelectric-like factor).
_TISSUES = {
    "air": (0.0012, 0.9),
    "water": (1.00, 1.0),
    "lung": (0.35, 1.0),
    "compact_bone": (1.85, 5.0),
    "cortical_bone": (1.92, 6.5),
    "cancellous_bone": (1.18, 2.5),
    "adipose": (0.95, 0.55),
    "brain": (1.04, 1.05),
    "b100": (1.45, 3.5),
    "skin": (1.09, 1.0),
    "muscle": (1.05, 1.05),
    "grey_matter": (1.04, 1.08),
    "white_matter": (1.04, 1.0),
    "csf": (1.01, 1.0),
    "blood": (1.06, 1.12),
}


def material_tables(rng: np.random.Generator, names: Sequence[str], energies: np.ndarray,
                    e_ref: float, base: tuple[float, float, float],
                    weights: np.ndarray, chord_mm: float, target_depth: float) -> np.ndarray:
    """mu[m][e] = rho_m * (a_m (E/E_ref)^-3 + b_m (E/E_ref)^-beta_m + c_m) in mm^-1.

    Smooth, positive, decreasing power laws.  The water-like material's
    optical depth along ``chord_mm`` at the ``weights``-averaged energy is
    calibrated to ``target_depth``; every material is scaled by the same
    factor.
    """
    a0, b0, c0 = base
    x = energies / e_ref
    rows = []
    for name in names:
        rho, photo = _TISSUES[name]
        j = 1.0 + 0.05 * np.clip(rng.standard_normal(3), -2.0, 2.0)
        beta = rng.uniform(0.2, 0.6)
        a = a0 * photo * j[0]
        b = b0 * j[1]
        c = c0 * j[2]
        rows.append(rho * (a * x ** -3.0 + b * x ** -beta + c))
    mu = np.array(rows, dtype=np.float64)
    e_mean = float(np.sum(weights * energies) / np.sum(weights))
    ref_name = "water" if "water" in names else ("brain" if "brain" in names else names[1])
    w_idx = list(names).index(ref_name)
    mu_ref = float(np.interp(e_mean, energies, mu[w_idx]))
    scale = target_depth / (mu_ref * chord_mm)
    return (mu * scale).astype(np.float32)


def kramers_spectrum(rng: np.random.Generator, energies: np.ndarray, e_max: float,
                     e_ref: float, tau_range: tuple[float, float]) -> np.ndarray:
    """phi(E) ~ max(0, Emax-E)/E * exp(-tau (E/Eref)^-3) * (1 + 0.05 sum_k c_k cos(k pi E/Emax)), sum 1."""
    tau = rng.uniform(*tau_range)
    ck = rng.standard_normal(3)
    ripple = 1.0 + 0.05 * sum(ck[k - 1] * np.cos(k * np.pi * energies / e_max) for k in (1, 2, 3))
    with np.errstate(over="ignore", under="ignore"):
        phi = np.maximum(0.0, e_max - energies) / energies * np.exp(-tau * (energies / e_ref) ** -3.0) * ripple
    phi = np.maximum(phi, 0.0)
    return (phi / phi.sum()).astype(np.float32)


def detector_response(rng: np.random.Generator, energies: np.ndarray, e_ref: float) -> np.ndarray:
    """eta(E) = 1 - exp(-kappa (E/Eref)^-p), in (0, 1]."""
    kappa = rng.uniform(0.3, 1.5)
    p = rng.uniform(0.5, 1.5)
    eta = 1.0 - np.exp(-kappa * (energies / e_ref) ** -p)
    return np.clip(eta, 1e-6, 1.0).astype(np.float32)


def energy_absorption_ratio(rng: np.random.Generator, energies: np.ndarray, e_ref: float) -> np.ndarray:
    """A smooth water-like mu_en/mu(E) in (0, 1): high where absorption
    dominates at low energy, a dip in the Compton range, a slow rise above
    (made up for this synthetic stand-in; no database values)."""
    x = np.log(energies / e_ref)
    dip = rng.uniform(0.12, 0.2)
    width = rng.uniform(1.0, 1.6)
    low = 1.0 / (1.0 + np.exp(3.0 * (x + rng.uniform(0.8, 1.2))))
    rise = 0.55 / (1.0 + np.exp(-(x - rng.uniform(2.0, 3.0)) / width))
    r = dip + (0.9 - dip) * low + rise
    return np.clip(r, 0.05, 0.99).astype(np.float32)


def material_densities(names: Sequence[str]) -> np.ndarray:
    """Relative densities (g/cm^3) of the synthetic tissues, float64 [M]."""
    return np.array([_TISSUES[n][0] for n in names], dtype=np.float64)


def phantom_mass_kg(phantom: "Phantom", densities: np.ndarray) -> float:
    """Mass of the labelled phantom: voxel counts x density x voxel volume."""
    counts = np.bincount(phantom.labels.reshape(-1).astype(np.int64), minlength=densities.size)
    vox_cm3 = phantom.dx * phantom.dy * phantom.dz * 1e-3
    return float((counts[:densities.size] * densities).sum() * vox_cm3 * 1e-3)


def contiguous_groups(n_energy: int, n_groups: int) -> np.ndarray:
    """group_of_bin[e] = floor(e*G/E)."""
    return (np.arange(n_energy, dtype=np.int64) * n_groups // n_energy).astype(np.int32)


def refine_spectral(spec: "Spectral", factor: int) -> "Spectral":
    """The same source, attenuation and response on ``factor`` times finer bins.

    Each (uniform) bin is cut into ``factor`` equal sub-bins; mu and eta are
    interpolated linearly at the sub-bin centres (held constant beyond the
    end centres), phi likewise and renormalised to sum 1, and the groups
    stay contiguous over the new bins (so each group keeps its energy range).
    """
    e = np.asarray(spec.energies, np.float64)
    step = (e[-1] - e[0]) / (e.size - 1)
    sub = (np.arange(factor) + 0.5) / factor - 0.5
    ef = (e[:, None] + sub[None, :] * step).ravel()
    mu = np.stack([np.interp(ef, e, np.asarray(row, np.float64)) for row in spec.mu]).astype(np.float32)
    phi = np.interp(ef, e, np.asarray(spec.phi, np.float64))
    eta = np.interp(ef, e, np.asarray(spec.eta, np.float64)).astype(np.float32)
    return Spectral(energies=ef, mu=mu, phi=(phi / phi.sum()).astype(np.float32), eta=eta,
                    n_groups=spec.n_groups, group_of_bin=contiguous_groups(ef.size, spec.n_groups),
                    flood=spec.flood, energy_unit=spec.energy_unit, material_names=spec.material_names)


def gaussian_psfs(rng: np.random.Generator, n_groups: int, k: int,
                  sigma_range: tuple[float, float] = (0.5, 2.0)) -> np.ndarray:
    """Rotated anisotropic Gaussians with a sub-pixel centre offset, each summing to 1.

    The rotation and offset make every kernel asymmetric and non-separable,
    so a convolution that forgets to flip the kernel, or assumes a
    separable kernel, gives a different answer.
    """
    c = (k - 1) / 2.0
    yy, xx = np.mgrid[0:k, 0:k].astype(np.float64)
    sig_major = np.sort(rng.uniform(*sigma_range, size=n_groups))
    out = np.empty((n_groups, k, k), dtype=np.float32)
    for g in range(n_groups):
        s1 = sig_major[g]
        s2 = s1 * rng.uniform(0.7, 1.0)
        rot = rng.uniform(0.0, np.pi)
        ox, oy = rng.uniform(-0.25, 0.25, size=2)
        x = xx - c - ox
        y = yy - c - oy
        xr = np.cos(rot) * x + np.sin(rot) * y
        yr = -np.sin(rot) * x + np.cos(rot) * y
        ker = np.exp(-0.5 * ((xr / s1) ** 2 + (yr / s2) ** 2))
        out[g] = (ker / ker.sum()).astype(np.float32)
    return out


def scatter_blobs(rng: np.random.Generator, n_angles: int, nu: int, nv: int,
                  sigma_u: tuple[float, float], sigma_v: tuple[float, float],
                  amp: tuple[float, float] = (0.05, 0.20), jitter: float = 20.0) -> Scatter:
    return Scatter(
        nu=nu, nv=nv,
        amp=rng.uniform(*amp, size=n_angles),
        cu=(nu - 1) / 2.0 + rng.uniform(-jitter, jitter, size=n_angles),
        cv=(nv - 1) / 2.0 + rng.uniform(-jitter, jitter, size=n_angles) * (nv / 64.0),
        su=rng.uniform(*sigma_u, size=n_angles),
        sv=rng.uniform(*sigma_v, size=n_angles),
    )


# ------------------------------------------------------------------ phantoms

def _centres(n: int, h: float, c: float) -> np.ndarray:
    return c - n * h / 2.0 + (np.arange(n, dtype=np.float64) + 0.5) * h


def cylinder_phantom(nx: int, ny: int, nz: int, h_xy: float, h_z: float, radius: float,
                     inserts: Sequence[tuple[float, float, float, int]]) -> np.ndarray:
    """Full-height water cylinder (label 1) in air (label 0) with cylindrical inserts.

    ``inserts`` holds (x_centre, y_centre, radius, label).  A voxel belongs to
    a body when its centre lies inside it.
    """
    x = _centres(nx, h_xy, 0.0)
    y = _centres(ny, h_xy, 0.0)
    lab2 = np.zeros((ny, nx), dtype=np.int8)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    lab2[r2 <= radius * radius] = 1
    for (xc, yc, r, label) in inserts:
        i0 = max(0, int(np.floor((xc - r - x[0]) / h_xy)) - 1)
        i1 = min(nx, int(np.ceil((xc + r - x[0]) / h_xy)) + 2)
        j0 = max(0, int(np.floor((yc - r - y[0]) / h_xy)) - 1)
        j1 = min(ny, int(np.ceil((yc + r - y[0]) / h_xy)) + 2)
        sub = (x[None, i0:i1] - xc) ** 2 + (y[j0:j1, None] - yc) ** 2 <= r * r
        lab2[j0:j1, i0:i1][sub] = label
    return np.ascontiguousarray(np.broadcast_to(lab2, (nz, ny, nx))).astype(np.int8)


def ellipsoid_phantom(nx: int, ny: int, nz: int, h: float,
                      bodies: Sequence[tuple[tuple[float, float, float], tuple[float, float, float], int]]) -> np.ndarray:
    """Paint ellipsoids (centre, semi-axes, label) in order onto an air volume."""
    x = _centres(nx, h, 0.0).astype(np.float32)
    y = _centres(ny, h, 0.0).astype(np.float32)
    z = _centres(nz, h, 0.0)
    lab = np.zeros((nz, ny, nx), dtype=np.int8)
    for iz in range(nz):
        sl = lab[iz]
        for (c, s, label) in bodies:
            dzn = (z[iz] - c[2]) / s[2]
            rest = 1.0 - dzn * dzn
            if rest < 0.0:
                continue
            m = ((x[None, :] - c[0]) / s[0]) ** 2 + ((y[:, None] - c[1]) / s[1]) ** 2 <= rest
            sl[m] = label
    return lab


def random_phantom(rng: np.random.Generator, nx: int, ny: int, nz: int, n_mat: int) -> np.ndarray:
    """Independent uniform labels in 0..n_mat-1 (for brute-force checks on tiny volumes)."""
    return rng.integers(0, n_mat, size=(nz, ny, nx)).astype(np.int8)


# ------------------------------------------------------------- configurations
#
# Each configuration is described by a JSON file in synth/configs/ (geometry,
# grid, seed, materials, energy bins, groups, optical-spread size, mode); the
# recipe named in the file builds the phantom's structure and the seeded
# tables.  make_config(n) loads the file of configuration n.

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")
CONFIG_FILES = {(1, ""): "tiny.json", (2, ""): "contrast.json", (2, "z"): "contrast_dz.json",
                (3, ""): "head.json", (4, ""): "contrast_split.json", (4, "z"): "contrast_dz.json",
                (5, ""): "head_surrogate.json"}


def _energies(p: dict) -> np.ndarray:
    e = p["energy"]
    return e["first"] + np.arange(e["bins"]) * (e["span"] / (e["bins"] - 1))


def _geometry(p: dict) -> Geometry:
    g = p["geometry"]
    return Geometry(sid=g["sid_mm"], sdd=g["sdd_mm"], nu=g["nu"], nv=g["nv"], du=g["du_mm"], dv=g["dv_mm"],
                    n_angles=g["n_angles"])


def _config1(rng: np.random.Generator, p: dict) -> Config:
    names, grid = p["materials"], p["grid"]
    energies = _energies(p)                                    # keV, bin centres
    phi = kramers_spectrum(rng, energies, 120.0, 30.0, (0.3, 0.6))
    eta = detector_response(rng, energies, 30.0)
    # water cylinder of 50 mm diameter (25 mm radius) so that air surrounds it
    ring = 12.0
    inserts = [(ring, 0.0, 2.0, 2), (0.0, ring, 3.0, 3), (-ring, 0.0, 4.0, 4), (0.0, -ring, 5.0, 5)]
    labels = cylinder_phantom(grid["nx"], grid["ny"], grid["nz"], grid["dx_mm"], grid["dz_mm"], 25.0, inserts)
    mu = material_tables(rng, names, energies, 30.0, (0.015, 0.015, 0.0075),
                         phi.astype(np.float64) * eta, 50.0, 3.0)
    spec = Spectral(energies=energies, mu=mu, phi=phi, eta=eta, n_groups=p["groups"],
                    group_of_bin=contiguous_groups(len(energies), p["groups"]), energy_unit=p["energy"]["unit"],
                    material_names=names)
    ph = Phantom(dx=grid["dx_mm"], dy=grid["dy_mm"], dz=grid["dz_mm"], labels=labels)
    return Config(p["name"], _geometry(p), ph, spec, None, None)


def _config2(rng: np.random.Generator, p: dict) -> Config:
    names, grid, g = p["materials"], p["grid"], p["geometry"]
    energies = _energies(p)                                    # MeV, bin centres
    phi = kramers_spectrum(rng, energies, 6.0, 1.0, (0.01, 0.03))
    eta = detector_response(rng, energies, 1.0)
    h = grid["dx_mm"]
    inserts = []
    diam = [1.0, 2.0, 3.0, 4.0, 5.0]
    radii = [30.0, 37.5, 45.0, 52.5, 60.0]
    for t in range(6):                     # one tissue per 60-degree sector
        for k in range(5):
            ang = np.deg2rad(60.0 * t + 12.0 * k + 6.0 + rng.uniform(-3.0, 3.0))
            r = radii[k] + rng.uniform(-2.0, 2.0)
            inserts.append((r * np.cos(ang), r * np.sin(ang), diam[k] / 2.0, 2 + t))
    labels = cylinder_phantom(grid["nx"], grid["ny"], grid["nz"], h, grid["dz_mm"], 80.0, inserts)
    mu = material_tables(rng, names, energies, 1.0, (5.0e-6, 0.05, 0.02),
                         phi.astype(np.float64) * eta, 160.0, 1.0)
    spec = Spectral(energies=energies, mu=mu, phi=phi, eta=eta, n_groups=p["groups"],
                    group_of_bin=contiguous_groups(len(energies), p["groups"]), energy_unit=p["energy"]["unit"],
                    material_names=names)
    ph = Phantom(dx=h, dy=grid["dy_mm"], dz=grid["dz_mm"], labels=labels)
    sc = scatter_blobs(rng, g["n_angles"], g["nu"], g["nv"], (200.0, 300.0), (30.0, 60.0)) if p["scatter"] else None
    psf = Psf(gaussian_psfs(rng, p["groups"], p["psf_k"])) if p["psf_k"] else None
    return Config(p["name"], _geometry(p), ph, spec, sc, psf)


def _config3(rng: np.random.Generator, p: dict) -> Config:
    names, grid, g = p["materials"], p["grid"], p["geometry"]
    energies = _energies(p)                                    # keV, 1-keV bins
    phi = kramers_spectrum(rng, energies, 120.0, 30.0, (0.3, 0.6))
    eta = detector_response(rng, energies, 30.0)
    j = lambda s: 1.0 + s * rng.uniform(-1.0, 1.0)
    a, b, c = 75.0 * j(0.04), 95.0 * j(0.04), 58.0 * j(0.04)
    cz0 = rng.uniform(-3.0, 3.0)
    shell = lambda t: ((0.0, 0.0, cz0), (a - t, b - t, c - t))
    bodies = [
        (*shell(0.0), 1),        # skin
        (*shell(2.0), 2),        # subcutaneous fat
        (*shell(4.5), 4),        # outer cortical table
        (*shell(6.5), 5),        # diploe
        (*shell(9.0), 4),        # inner cortical table
        (*shell(11.0), 6),       # grey matter
        (*shell(15.0), 7),       # white matter
        ((0.0, 8.0, cz0 - 40.0), (48.0, 55.0, 22.0), 3),          # jaw / neck muscle
    ]
    for sgn in (-1.0, 1.0):     # lateral ventricles
        bodies.append(((sgn * (7.0 + rng.uniform(-1, 1)), rng.uniform(-5, 5), cz0 + 8.0),
                       (4.5, 20.0 * j(0.1), 9.0 * j(0.1)), 8))
    bodies.append(((0.0, -20.0, cz0 + 5.0), (2.0, 25.0, 2.0), 9))       # a vessel-like tube
    bodies.append(((0.0, 0.0, cz0 + 48.0), (3.0, 70.0, 3.0), 9))        # sagittal-sinus-like tube
    for sgn in (-1.0, 1.0):     # air sinuses
        bodies.append(((sgn * 14.0, 78.0 * j(0.03), cz0 - 22.0), (9.0, 7.0, 8.0), 0))
    labels = ellipsoid_phantom(grid["nx"], grid["ny"], grid["nz"], grid["dx_mm"], bodies)
    mu = material_tables(rng, names, energies, 30.0, (0.015, 0.015, 0.0075),
                         phi.astype(np.float64) * eta, 2.0 * a, 3.0)
    spec = Spectral(energies=energies, mu=mu, phi=phi, eta=eta, n_groups=p["groups"],
                    group_of_bin=contiguous_groups(len(energies), p["groups"]), energy_unit=p["energy"]["unit"],
                    material_names=names)
    ph = Phantom(dx=grid["dx_mm"], dy=grid["dy_mm"], dz=grid["dz_mm"], labels=labels)
    sc = scatter_blobs(rng, g["n_angles"], g["nu"], g["nv"], (200.0, 300.0), (360.0, 720.0)) if p["scatter"] else None
    psf = Psf(gaussian_psfs(rng, p["groups"], p["psf_k"])) if p["psf_k"] else None
    return Config(p["name"], _geometry(p), ph, spec, sc, psf)


RECIPES = {"tiny": _config1, "contrast": _config2, "head": _config3}


def load_config(source) -> Config:
    """A configuration from a JSON file (path) or its parsed dict: the recipe
    builds the phantom and the seeded tables with the file's geometry, grid,
    seed, materials, energy bins, groups and optical-spread size; ``mode``
    names the projector form it is meant for."""
    p = source if isinstance(source, dict) else json.load(open(source))
    if p.get("recipe") not in RECIPES:
        raise ValueError(f"unknown recipe {p.get('recipe')!r}; known: {sorted(RECIPES)}")
    cfg = RECIPES[p["recipe"]](np.random.default_rng(int(p["seed"])), p)
    cfg.mode = p.get("mode", "plain")
    return cfg


def make_config(n: int, variant: str = "") -> Config:
    """Configuration ``n`` (1 tiny, 2 contrast, 3 head, 4 = 2 split, 5 = 3 surrogate).

    ``variant="z"`` with n in (2, 4) gives the thick-slab contrast phantom
    (dz = 1.5625 mm, the ten slices fill the 64-row cone).
    """
    key = (int(n), variant)
    if key not in CONFIG_FILES:
        raise ValueError(f"no configuration {n}{' variant ' + variant if variant else ''}")
    cfg = load_config(os.path.join(CONFIG_DIR, CONFIG_FILES[key]))
    if key == (4, "z"):
        cfg.mode = "split_bf16"
    return cfg
