"""FP64 CPU oracle for the polyenergetic cone-beam projector (fastCAT, arXiv 2011.04736).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it, and it shares no code with the HIP path: the arithmetic lives
in ``fcat_oracle.c`` (plain C, FP64, OpenMP over rays) and in ``mlp.py``
(NumPy FP64); this module only converts arrays and calls it.

Functions and the passages they follow:

* ``siddon`` / ``pathlengths`` / ``pathlengths_rays`` -- Sec. II.F: a
  projection is the line integral of the attenuation along the ray; with the
  labelled phantom of Sec. II.C that integral is sum_m mu_m(E) L_m, so the
  oracle computes the per-material path lengths L_m exactly (Siddon 1985,
  merged parametric plane crossings).
* ``bruteforce`` -- an independent midpoint-rule sampler of the same L_m.
* ``spectral`` -- Eq. 3 with the scatter added to the primary profiles
  before the spectrum x response weighting (Sec. II.F).
* ``psf`` -- Sec. II.G: convolution of each group's profile with its optical
  spread kernel (Eq. 1 normalisation), then the sum over groups.
* ``project`` -- all of the above for a list of angles.
* ``forward_image`` / ``backproject_image`` -- the projector of a real-valued
  voxel image (the Sec. II.F line integral over an image, as an iterative
  reconstruction of Sec. II.G needs it) and its transpose, from the same
  Siddon segments: (A f)_r = sum_k l_rk f_k and (A^T y)_k = sum_r l_rk y_r.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcat_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libfcat_oracle.so")
_lock = threading.Lock()
_lib = None

OK, BAD_LABEL, NOMEM, BAD_ARG = 0, 1, 2, 3


class _Geometry(C.Structure):
    _fields_ = [("sid", C.c_double), ("sdd", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double),
                ("off_u", C.c_double), ("off_v", C.c_double),
                ("n_angles", C.c_int32),
                ("angles", C.POINTER(C.c_double))]


class _Volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double),
                ("labels", C.POINTER(C.c_int8))]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-fno-fast-math", "-ffp-contract=off", "-D_DEFAULT_SOURCE",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib() -> C.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB_PATH)
            dp = C.POINTER(C.c_double)
            gp = C.POINTER(_Geometry)
            vp = C.POINTER(_Volume)
            i32p = C.POINTER(C.c_int32)
            i64p = C.POINTER(C.c_int64)
            L.orc_siddon.argtypes = [dp, dp, vp, C.c_int, dp]
            L.orc_bruteforce.argtypes = [dp, dp, vp, C.c_int, C.c_int64, dp]
            L.orc_ray_endpoints.argtypes = [gp, C.c_int, C.c_int, C.c_int, dp, dp]
            L.orc_ray_endpoints.restype = None
            L.orc_angle.argtypes = [gp, C.c_int]
            L.orc_angle.restype = C.c_double
            L.orc_pathlengths_rays.argtypes = [gp, vp, C.c_int, i64p, C.c_int64, dp, C.c_int]
            L.orc_pathlengths.argtypes = [gp, vp, C.c_int, i32p, C.c_int, dp, C.c_int]
            L.orc_spectral.argtypes = [dp, C.c_int64, C.c_int, C.c_int, C.c_int, dp, dp, dp, i32p,
                                       dp, dp, dp, dp, C.c_int]
            L.orc_spectral.restype = None
            L.orc_psf.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_int, dp, C.c_int]
            L.orc_psf.restype = None
            L.orc_project.argtypes = [gp, vp, C.c_int, C.c_int, C.c_int, dp, dp, dp, i32p,
                                      dp, dp, dp, dp, C.c_int, i32p, C.c_int, dp, dp, C.c_int]
            L.orc_max_threads.argtypes = []
            grp = C.POINTER(_Grid)
            L.orc_forward_image.argtypes = [gp, grp, dp, i32p, C.c_int, dp, C.c_int]
            L.orc_backproject_image.argtypes = [gp, grp, dp, i32p, C.c_int, dp, C.c_int]
            _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ------------------------------------------------------------------ helpers

def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Keep:
    """Holds the NumPy arrays a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def add(self, a):
        self.refs.append(a)
        return a


def _geom(g, keep: _Keep) -> _Geometry:
    ang = None if g.angles is None else keep.add(_f64(g.angles))
    return _Geometry(float(g.sid), float(g.sdd), int(g.nu), int(g.nv), float(g.du), float(g.dv),
                     float(g.off_u), float(g.off_v), int(g.n_angles),
                     _dptr(ang))


def _vol(p, keep: _Keep) -> _Volume:
    lab = keep.add(np.ascontiguousarray(p.labels, dtype=np.int8))
    nz, ny, nx = lab.shape
    return _Volume(nx, ny, nz, float(p.dx), float(p.dy), float(p.dz),
                   float(p.cx), float(p.cy), float(p.cz),
                   lab.ctypes.data_as(C.POINTER(C.c_int8)))


def _check(rc: int, what: str):
    if rc == BAD_LABEL:
        raise ValueError(f"{what}: a label is outside 0..n_mat-1")
    if rc == NOMEM:
        raise MemoryError(what)
    if rc != OK:
        raise RuntimeError(f"{what}: status {rc}")


# ------------------------------------------------------------ path lengths

def siddon(src, dst, phantom, n_mat: int) -> np.ndarray:
    """Exact per-material length of segment src->dst (Siddon 1985)."""
    keep = _Keep()
    v = _vol(phantom, keep)
    s, d = _f64(src), _f64(dst)
    L = np.zeros(n_mat, dtype=np.float64)
    _check(lib().orc_siddon(_dptr(s), _dptr(d), C.byref(v), n_mat, _dptr(L)), "siddon")
    return L


def bruteforce(src, dst, phantom, n_mat: int, n_steps: int = 1_000_000) -> np.ndarray:
    """Midpoint-rule per-material lengths with n_steps equal steps over src->dst."""
    keep = _Keep()
    v = _vol(phantom, keep)
    s, d = _f64(src), _f64(dst)
    L = np.zeros(n_mat, dtype=np.float64)
    _check(lib().orc_bruteforce(_dptr(s), _dptr(d), C.byref(v), n_mat, int(n_steps), _dptr(L)),
           "bruteforce")
    return L


def ray_endpoints(geometry, a: int, iv: int, iu: int):
    keep = _Keep()
    g = _geom(geometry, keep)
    s = np.zeros(3)
    p = np.zeros(3)
    lib().orc_ray_endpoints(C.byref(g), int(a), int(iv), int(iu), _dptr(s), _dptr(p))
    return s, p


def pathlengths_rays(geometry, phantom, n_mat: int, ray_ids, n_threads: int = 0) -> np.ndarray:
    """L[n][M] for rays with id (a*nv + iv)*nu + iu."""
    keep = _Keep()
    g, v = _geom(geometry, keep), _vol(phantom, keep)
    ids = np.ascontiguousarray(np.asarray(ray_ids, dtype=np.int64).reshape(-1))
    L = np.zeros((ids.size, n_mat), dtype=np.float64)
    _check(lib().orc_pathlengths_rays(C.byref(g), C.byref(v), n_mat,
                                      ids.ctypes.data_as(C.POINTER(C.c_int64)), ids.size,
                                      _dptr(L), n_threads), "pathlengths_rays")
    return L


def pathlengths(geometry, phantom, n_mat: int, angle_idx: Sequence[int], n_threads: int = 0) -> np.ndarray:
    """L[n_ang][nv][nu][M] for every pixel of the listed angles."""
    keep = _Keep()
    g, v = _geom(geometry, keep), _vol(phantom, keep)
    ai = np.ascontiguousarray(np.asarray(angle_idx, dtype=np.int32).reshape(-1))
    L = np.zeros((ai.size, geometry.nv, geometry.nu, n_mat), dtype=np.float64)
    _check(lib().orc_pathlengths(C.byref(g), C.byref(v), n_mat,
                                 ai.ctypes.data_as(C.POINTER(C.c_int32)), ai.size,
                                 _dptr(L), n_threads), "pathlengths")
    return L


# ------------------------------------------------------------ spectral, psf

def spectral(L, mu, phi, eta, group_of_bin, n_groups: int, i0=None, S=None, s_bin=None,
             n_threads: int = 0) -> np.ndarray:
    """Y[G][n] = sum_{e in g} phi_e eta_e (I0 exp(-sum_m mu[m][e] L[m]) + s_e S)  (Eq. 3)."""
    L = _f64(L)
    n_mat = L.shape[-1]
    L2 = L.reshape(-1, n_mat)
    n = L2.shape[0]
    mu = _f64(mu)
    n_energy = mu.shape[1]
    grp = np.ascontiguousarray(np.asarray(group_of_bin, dtype=np.int32))
    i0a = None if i0 is None else _f64(i0).reshape(-1)
    Sa = None if S is None else _f64(S).reshape(-1)
    sb = _f64(s_bin)
    Y = np.zeros((n_groups, n), dtype=np.float64)
    lib().orc_spectral(_dptr(L2), n, n_mat, n_energy, n_groups, _dptr(mu), _dptr(_f64(phi)),
                       _dptr(_f64(eta)), grp.ctypes.data_as(C.POINTER(C.c_int32)),
                       _dptr(i0a), _dptr(Sa), _dptr(sb), _dptr(Y), n_threads)
    return Y


def psf(Y, kernels, n_threads: int = 0) -> np.ndarray:
    """out[a][v][u] = sum_g (K_g * Y[a][g])[v][u], zero-padded same-size convolution."""
    Y = _f64(Y)
    n_ang, n_groups, nv, nu = Y.shape
    K = _f64(kernels)
    k = K.shape[-1]
    out = np.zeros((n_ang, nv, nu), dtype=np.float64)
    lib().orc_psf(_dptr(Y), n_ang, n_groups, nv, nu, _dptr(K), k, _dptr(out), n_threads)
    return out


def project(cfg, angle_idx: Sequence[int], with_groups: bool = False, scatter: bool = True,
            use_psf: bool = True, n_threads: int = 0, scatter_maps=None):
    """FP64 projections out[n_ang][nv][nu] of the listed angles of a configuration.

    With ``with_groups`` also returns the group signals Y[n_ang][G][nv][nu]
    before the optical spread.
    """
    keep = _Keep()
    geo, ph, sp = cfg.geometry, cfg.phantom, cfg.spectral
    g, v = _geom(geo, keep), _vol(ph, keep)
    ai = np.ascontiguousarray(np.asarray(angle_idx, dtype=np.int32).reshape(-1))
    n_ang = ai.size
    mu, phi, eta = _f64(sp.mu), _f64(sp.phi), _f64(sp.eta)
    grp = np.ascontiguousarray(np.asarray(sp.group_of_bin, dtype=np.int32))
    flood = None if sp.flood is None else _f64(sp.flood)
    S = None
    sb = None
    if scatter and cfg.scatter is not None:
        S = _f64(cfg.scatter.maps(ai) if scatter_maps is None else scatter_maps)
        sb = _f64(cfg.scatter.s_bin)
    K = None
    k = 1
    if use_psf and cfg.psf is not None:
        K = _f64(cfg.psf.kernels)
        k = K.shape[-1]
    out = np.zeros((n_ang, geo.nv, geo.nu), dtype=np.float64)
    Y = np.zeros((n_ang, sp.n_groups, geo.nv, geo.nu), dtype=np.float64) if with_groups else None
    rc = lib().orc_project(C.byref(g), C.byref(v), sp.n_mat, sp.n_energy, sp.n_groups,
                           _dptr(mu), _dptr(phi), _dptr(eta), grp.ctypes.data_as(C.POINTER(C.c_int32)),
                           _dptr(flood), _dptr(S), _dptr(sb), _dptr(K), k,
                           ai.ctypes.data_as(C.POINTER(C.c_int32)), n_ang, _dptr(out), _dptr(Y), n_threads)
    _check(rc, "project")
    return (out, Y) if with_groups else out


# ------------------------------------------------------- image projector pair

def _cgrid(grid) -> _Grid:
    return _Grid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx), float(grid.dy), float(grid.dz),
                 float(getattr(grid, "cx", 0.0)), float(getattr(grid, "cy", 0.0)), float(getattr(grid, "cz", 0.0)))


def forward_image(geometry, grid, image, angle_idx: Sequence[int], n_threads: int = 0) -> np.ndarray:
    """(A f)[n_ang][nv][nu]: line integrals of image [nz][ny][nx] over the grid."""
    keep = _Keep()
    g, gr = _geom(geometry, keep), _cgrid(grid)
    f = _f64(image)
    assert f.shape == (grid.nz, grid.ny, grid.nx)
    ai = np.ascontiguousarray(np.asarray(angle_idx, dtype=np.int32).reshape(-1))
    out = np.zeros((ai.size, geometry.nv, geometry.nu), np.float64)
    _check(lib().orc_forward_image(C.byref(g), C.byref(gr), _dptr(f), ai.ctypes.data_as(C.POINTER(C.c_int32)),
                                   ai.size, _dptr(out), n_threads), "forward_image")
    return out


def backproject_image(geometry, grid, proj, angle_idx: Sequence[int], n_threads: int = 0) -> np.ndarray:
    """(A^T y)[nz][ny][nx] for y = proj [n_ang][nv][nu] of the listed angles."""
    keep = _Keep()
    g, gr = _geom(geometry, keep), _cgrid(grid)
    y = _f64(proj)
    ai = np.ascontiguousarray(np.asarray(angle_idx, dtype=np.int32).reshape(-1))
    assert y.shape == (ai.size, geometry.nv, geometry.nu)
    img = np.zeros((grid.nz, grid.ny, grid.nx), np.float64)
    _check(lib().orc_backproject_image(C.byref(g), C.byref(gr), _dptr(y), ai.ctypes.data_as(C.POINTER(C.c_int32)),
                                       ai.size, _dptr(img), n_threads), "backproject_image")
    return img
