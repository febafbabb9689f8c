"""MI355X-native polyenergetic cone-beam projector (fastCAT, arXiv 2011.04736).

Thin Python binding of ``libfcat.so`` (C ABI in ``include/fcat.h``).  Every
step of the projector runs in the library's HIP kernels; this module only
marshals arguments: it builds the C descriptors from device tensors, passes
``data_ptr()`` values and the current HIP stream, allocates outputs and
workspaces with PyTorch, and turns non-OK status codes into ``FcatError``.

The functions keep the C names (``fcat_project``, ``fcat_pathlengths``,
``fcat_spectral``, ``fcat_psf``, ``fcat_check_inputs`` ...).  ``upload``
moves a host-side problem description (geometry, labelled phantom, spectral
tables, optional scatter maps and optical spread kernels) to the GPU.

If the library has not been built, or no GPU is present, the entry points
raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import functools
import math
import os
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "FcatError", "MODES", "STAGES", "Geometry", "Phantom", "Spectral", "Scatter", "Psf", "Problem", "Noise",
    "Surrogate", "MlpTrain", "lib_path", "load", "upload", "project", "fcat_version", "fcat_status_string",
    "fcat_last_error", "fcat_project_workspace_bytes", "fcat_project", "fcat_project_status", "fcat_pathlengths_workspace_bytes",
    "fcat_pathlengths", "fcat_walk_stats", "WALK_COUNTS", "fcat_spectral_workspace_bytes", "fcat_spectral", "fcat_spectral_static", "fcat_psf", "fcat_check_inputs",
    "fcat_timing_enable", "fcat_timing_read", "fcat_count_scale", "fcat_poisson", "fcat_flood_workspace_bytes",
    "fcat_flood_profile", "fcat_log_projection", "fcat_projections_workspace_bytes", "fcat_projections",
    "fcat_dose_workspace_bytes", "fcat_dose", "fcat_fdk_filter", "fcat_fdk_backproject_workspace_bytes",
    "fcat_fdk_backproject", "fcat_fdk_workspace_bytes", "fcat_fdk", "fcat_image_project", "fcat_image_backproject", "fcat_effective_psf",
    "fcat_slit_lsf_range", "fcat_slit_mtf", "fcat_richardson_lucy_workspace_bytes",
    "fcat_slit_mtf_workspace_bytes", "fcat_richardson_lucy", "fcat_mlp_param_count",
    "fcat_mlp_workspace_bytes", "fcat_mlp_linear_term", "fcat_mlp_forward", "fcat_mlp_gradients",
    "fcat_mlp_train_step", "fcat_mlp_train_epoch", "fcat_mlp_validate", "fcat_mlp_setup",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfcat.so")
MODES = {"plain": 0, "split_bf16": 1, "surrogate": 2}
STAGES = ("prep", "trace", "psf", "mlp", "noise", "proj", "dose", "filter", "backproject", "optics", "layout")
_lib = None


class FcatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fcat status {status}: {message}")
        self.status = status


# ------------------------------------------------------------ C structures

class _CGeometry(C.Structure):
    _fields_ = [("sid_mm", C.c_double), ("sdd_mm", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du_mm", C.c_double), ("dv_mm", C.c_double),
                ("off_u_mm", C.c_double), ("off_v_mm", C.c_double),
                ("n_angles", C.c_int32), ("angles_rad", C.c_void_p)]


class _CPhantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx_mm", C.c_double), ("dy_mm", C.c_double), ("dz_mm", C.c_double),
                ("cx_mm", C.c_double), ("cy_mm", C.c_double), ("cz_mm", C.c_double),
                ("labels", C.c_void_p)]


class _CSpectral(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("n_energy", C.c_int32), ("n_groups", C.c_int32),
                ("mu", C.c_void_p), ("phi", C.c_void_p), ("eta", C.c_void_p),
                ("flood", C.c_void_p), ("group_of_bin", C.POINTER(C.c_int32))]


class _CScatter(C.Structure):
    _fields_ = [("maps", C.c_void_p), ("s_bin", C.c_void_p)]


class _CPsf(C.Structure):
    _fields_ = [("k", C.c_int32), ("kernels", C.c_void_p)]


class _CGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx_mm", C.c_double), ("dy_mm", C.c_double), ("dz_mm", C.c_double),
                ("cx_mm", C.c_double), ("cy_mm", C.c_double), ("cz_mm", C.c_double)]


class _CNoise(C.Structure):
    _fields_ = [("counts_per_pixel", C.c_double), ("seed", C.c_uint64), ("floor", C.c_float)]


class _CSurrogate(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_out", C.c_int32), ("params", C.c_void_p),
                ("in_scale", C.c_void_p), ("out_scale", C.c_void_p), ("lin", C.c_void_p), ("cell_ok", C.c_void_p),
                ("cell_lo", C.c_float), ("cell_hi", C.c_float), ("counts", C.c_void_p)]


class _CTrain(C.Structure):
    _fields_ = [("params", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("step", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


def lib_path() -> str:
    return _LIB_PATH


def load() -> C.CDLL:
    """Load libfcat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run __graft_entry__.build() "
                          f"or python -m paper_2011_04736_amd._build")
    # PyTorch bundles its own HIP runtime with the same soname as ROCm's.  Load
    # it first so that libfcat.so binds to that one instance: two runtimes in
    # one process would each try to own the device.
    import torch  # noqa: F401
    L = C.CDLL(_LIB_PATH)
    vp, sz, st = C.c_void_p, C.c_size_t, C.c_int
    gp, pp, sp = C.POINTER(_CGeometry), C.POINTER(_CPhantom), C.POINTER(_CSpectral)
    scp, psp, sup = C.POINTER(_CScatter), C.POINTER(_CPsf), C.POINTER(_CSurrogate)
    L.fcat_version.restype = C.c_int
    L.fcat_status_string.argtypes = [st]
    L.fcat_status_string.restype = C.c_char_p
    L.fcat_last_error.restype = C.c_char_p
    L.fcat_project_workspace_bytes.argtypes = [gp, pp, sp, scp, psp, st, C.c_int32]
    L.fcat_project_workspace_bytes.restype = sz
    L.fcat_project.argtypes = [gp, pp, sp, scp, psp, st, sup, vp, vp, sz, vp]
    L.fcat_project.restype = st
    L.fcat_project_status.argtypes = [vp, sz, vp]
    L.fcat_project_status.restype = st
    L.fcat_pathlengths_workspace_bytes.argtypes = [pp]
    L.fcat_pathlengths_workspace_bytes.restype = sz
    L.fcat_pathlengths.argtypes = [gp, pp, C.c_int32, C.c_int32, C.c_int32, vp, vp, sz, vp]
    L.fcat_pathlengths.restype = st
    L.fcat_walk_stats.argtypes = [gp, pp, C.c_int32, C.c_int32, vp, vp, sz, vp]
    L.fcat_walk_stats.restype = st
    L.fcat_spectral_workspace_bytes.argtypes = [sp]
    L.fcat_spectral_workspace_bytes.restype = sz
    L.fcat_spectral.argtypes = [vp, C.c_int64, sp, vp, vp, vp, st, vp, vp, sz, vp]
    L.fcat_spectral.restype = st
    L.fcat_spectral_static.argtypes = [vp, C.c_int64, sp, vp, vp, vp, st, vp, vp]
    L.fcat_spectral_static.restype = st
    L.fcat_psf.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, psp, vp, vp]
    L.fcat_psf.restype = st
    L.fcat_check_inputs.argtypes = [gp, pp, sp, scp, psp, vp, sz, vp]
    L.fcat_check_inputs.restype = st
    sup2, trp = C.POINTER(_CSurrogate), C.POINTER(_CTrain)
    i64 = C.c_int64
    L.fcat_mlp_param_count.argtypes = [C.c_int32, C.c_int32]
    L.fcat_mlp_param_count.restype = C.c_int32
    L.fcat_mlp_workspace_bytes.argtypes = [sp, i64]
    L.fcat_mlp_workspace_bytes.restype = sz
    L.fcat_mlp_linear_term.argtypes = [sp, vp, vp, sz, vp]
    L.fcat_mlp_linear_term.restype = st
    L.fcat_mlp_forward.argtypes = [sup2, sp, vp, i64, vp, vp, sz, vp]
    L.fcat_mlp_forward.restype = st
    L.fcat_mlp_gradients.argtypes = [sup2, sp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.fcat_mlp_gradients.restype = st
    L.fcat_mlp_train_step.argtypes = [trp, sup2, sp, vp, vp, i64, vp, i64, C.c_int32, vp, vp, sz, vp]
    L.fcat_mlp_train_step.restype = st
    L.fcat_mlp_train_epoch.argtypes = [trp, sup2, sp, vp, vp, i64, vp, C.c_int32, vp, vp, sz, vp]
    L.fcat_mlp_train_epoch.restype = st
    L.fcat_mlp_validate.argtypes = [sup2, sp, vp, vp, i64, C.c_float, C.c_int32, vp, vp, vp, vp, sz, vp]
    L.fcat_mlp_validate.restype = st
    L.fcat_mlp_setup.argtypes = [sp, vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    L.fcat_mlp_setup.restype = st
    nzp, u64 = C.POINTER(_CNoise), C.c_uint64
    L.fcat_count_scale.argtypes = [sp, C.c_double, vp, vp]
    L.fcat_count_scale.restype = st
    L.fcat_poisson.argtypes = [vp, C.c_int32, C.c_int32, i64, vp, u64, C.c_int32, vp]
    L.fcat_poisson.restype = st
    L.fcat_flood_workspace_bytes.argtypes = [sp, C.c_int32, C.c_int32]
    L.fcat_flood_workspace_bytes.restype = sz
    L.fcat_flood_profile.argtypes = [sp, psp, C.c_int32, C.c_int32, vp, vp, sz, vp]
    L.fcat_flood_profile.restype = st
    L.fcat_log_projection.argtypes = [vp, vp, C.c_int32, i64, C.c_float, vp, vp]
    L.fcat_log_projection.restype = st
    L.fcat_projections_workspace_bytes.argtypes = [gp, pp, sp, scp, psp, st, C.c_int32]
    L.fcat_projections_workspace_bytes.restype = sz
    L.fcat_projections.argtypes = [gp, pp, sp, scp, psp, st, sup, nzp, vp, vp, sz, vp]
    L.fcat_projections.restype = st
    L.fcat_dose_workspace_bytes.argtypes = [gp, pp, sp, C.c_int32]
    L.fcat_dose_workspace_bytes.restype = sz
    L.fcat_dose.argtypes = [gp, pp, sp, vp, vp, C.c_double, C.c_int32, C.c_int32, vp, vp, vp, sz, vp]
    L.fcat_dose.restype = st
    grp = C.POINTER(_CGrid)
    L.fcat_fdk_filter.argtypes = [gp, vp, C.c_int32, vp, vp]
    L.fcat_fdk_filter.restype = st
    L.fcat_fdk_backproject_workspace_bytes.argtypes = [C.c_int32]
    L.fcat_fdk_backproject_workspace_bytes.restype = sz
    L.fcat_fdk_backproject.argtypes = [gp, vp, C.c_int32, C.c_int32, grp, vp, C.c_int32, vp, sz, vp]
    L.fcat_fdk_backproject.restype = st
    L.fcat_fdk_workspace_bytes.argtypes = [gp, C.c_int32]
    L.fcat_fdk_workspace_bytes.restype = sz
    L.fcat_fdk.argtypes = [gp, vp, grp, vp, vp, sz, vp]
    L.fcat_fdk.restype = st
    L.fcat_image_project.argtypes = [gp, grp, vp, C.c_int32, C.c_int32, vp, vp]
    L.fcat_image_project.restype = st
    L.fcat_image_backproject.argtypes = [gp, grp, vp, C.c_int32, C.c_int32, vp, C.c_int32, vp]
    L.fcat_image_backproject.restype = st
    L.fcat_effective_psf.argtypes = [sp, psp, vp, vp]
    L.fcat_effective_psf.restype = st
    L.fcat_slit_lsf_range.argtypes = [C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.fcat_slit_lsf_range.restype = st
    L.fcat_slit_mtf_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.fcat_slit_mtf_workspace_bytes.restype = sz
    L.fcat_slit_mtf.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                vp, C.c_int32, vp, vp, vp, vp, sz, vp]
    L.fcat_slit_mtf.restype = st
    L.fcat_richardson_lucy_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.fcat_richardson_lucy_workspace_bytes.restype = sz
    L.fcat_richardson_lucy.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32, C.c_int32, vp, vp, sz, vp]
    L.fcat_richardson_lucy.restype = st
    L.fcat_timing_enable.argtypes = [C.c_int]
    L.fcat_timing_enable.restype = st
    L.fcat_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32, C.c_int]
    L.fcat_timing_read.restype = st
    _lib = L
    return L


def _torch():
    import torch
    return torch


_noted = threading.local()


def _entry(fn):
    """Public entry point: starts a fresh list of the caller tensors whose
    device ``_require_gpu`` checks once every other argument check passed."""
    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        _noted.tensors = []
        return fn(*args, **kwargs)
    return wrapper


def _note(t, name: str):
    if not hasattr(_noted, "tensors"):
        _noted.tensors = []
    _noted.tensors.append((name, t))


def _require_gpu():
    """Raises ValueError for a noted caller tensor that is not on a GPU, then
    RuntimeError if no GPU is visible."""
    torch = _torch()
    for name, t in getattr(_noted, "tensors", []):
        if not t.is_cuda:
            raise ValueError(f"{name} must be on a GPU, not on {t.device}")
    _noted.tensors = []
    if not torch.cuda.is_available():
        raise RuntimeError("fcat needs a ROCm GPU (gfx950); none is visible")
    return torch


def _ptr(t) -> Optional[int]:
    """Pointer of a tensor this module allocated itself (no checks needed)."""
    if t is None:
        return None
    return int(t.data_ptr())


def _fmt_shape(shape) -> str:
    return "[" + "][".join("*" if d is None else str(d) for d in shape) + "]"


def _arg(t, name: str, dtype, shape=None, optional: bool = False) -> Optional[int]:
    """Device pointer of a caller's tensor, after the checks the C ABI cannot
    make: a torch.Tensor of ``dtype``, contiguous, of ``shape`` (a tuple whose
    None entries match any size), on a GPU.  ``None`` passes when optional.
    Raises ValueError, before anything reaches the library."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor, not {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and (t.dim() != len(shape) or
                              any(s is not None and int(d) != int(s) for d, s in zip(t.shape, shape))):
        raise ValueError(f"{name} must have shape {_fmt_shape(shape)}, not {list(t.shape)}")
    _note(t, name)
    return int(t.data_ptr())


def _ws(t, name: str = "workspace") -> tuple[Optional[int], int]:
    """(pointer, bytes) of a caller's workspace (any contiguous GPU tensor) or (None, 0)."""
    if t is None:
        return None, 0
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor, not {type(t).__name__}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    _note(t, name)
    return int(t.data_ptr()), int(t.numel() * t.element_size())


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check(status: int):
    if status != 0:
        lib = load()
        raise FcatError(status, f"{lib.fcat_status_string(status).decode()}: {lib.fcat_last_error().decode()}")


# ------------------------------------------------------------ descriptors

@dataclass
class Geometry:
    sid: float
    sdd: float
    nu: int
    nv: int
    du: float
    dv: float
    n_angles: int
    off_u: float = 0.0
    off_v: float = 0.0
    angles: object = None          # device float64 tensor [A] or None

    def c(self) -> _CGeometry:
        torch = _torch()
        ang = _arg(self.angles, "geometry.angles", torch.float64, (self.n_angles,), optional=True)
        return _CGeometry(self.sid, self.sdd, self.nu, self.nv, self.du, self.dv, self.off_u,
                          self.off_v, self.n_angles, ang)


@dataclass
class Phantom:
    labels: object                 # device int8 tensor [nz][ny][nx]
    dx: float
    dy: float
    dz: float
    cx: float = 0.0
    cy: float = 0.0
    cz: float = 0.0

    def c(self) -> _CPhantom:
        lab = _arg(self.labels, "phantom.labels", _torch().int8, (None, None, None))
        nz, ny, nx = self.labels.shape
        return _CPhantom(nx, ny, nz, self.dx, self.dy, self.dz, self.cx, self.cy, self.cz, lab)


@dataclass
class Spectral:
    mu: object                     # device float32 [M][E]
    phi: object                    # device float32 [E]
    eta: object                    # device float32 [E]
    n_groups: int
    group_of_bin: Optional[np.ndarray] = None   # host int32 [E] or None
    flood: object = None           # device float32 [nv][nu] or None

    def c(self) -> tuple[_CSpectral, object]:
        f32 = _torch().float32
        mu = _arg(self.mu, "spectral.mu", f32, (None, None))
        M, E = self.mu.shape
        phi = _arg(self.phi, "spectral.phi", f32, (E,))
        eta = _arg(self.eta, "spectral.eta", f32, (E,))
        flood = _arg(self.flood, "spectral.flood", f32, (None, None), optional=True)
        gob = None
        gptr = C.POINTER(C.c_int32)()
        if self.group_of_bin is not None:
            gob = np.ascontiguousarray(np.asarray(self.group_of_bin, dtype=np.int32))
            if gob.shape != (E,):
                raise ValueError(f"spectral.group_of_bin must have {E} entries, not {gob.shape}")
            gptr = gob.ctypes.data_as(C.POINTER(C.c_int32))
        return _CSpectral(M, E, self.n_groups, mu, phi, eta, flood, gptr), gob


@dataclass
class Scatter:
    maps: object                   # device float32 [A][nv][nu]
    s_bin: object = None           # device float32 [E] or None

    def c(self) -> _CScatter:
        f32 = _torch().float32
        return _CScatter(_arg(self.maps, "scatter.maps", f32, (None, None, None)),
                         _arg(self.s_bin, "scatter.s_bin", f32, (None,), optional=True))


@dataclass
class Psf:
    kernels: object                # device float32 [G][k][k]

    def c(self) -> _CPsf:
        ker = _arg(self.kernels, "psf.kernels", _torch().float32, (None, None, None))
        k = int(self.kernels.shape[-1])
        if int(self.kernels.shape[-2]) != k:
            raise ValueError(f"psf.kernels must be [G][k][k], not {list(self.kernels.shape)}")
        return _CPsf(k, ker)


@dataclass
class Surrogate:
    """Learned replacement of the primary spectral sum (device tensors)."""
    params: object                 # float32 [P]
    in_scale: object               # float32 [n_in]
    out_scale: object              # float32 [n_out]
    lin: object                    # float32 [n_out][n_in]
    cell_ok: object = None         # uint8 [n_in * 16]
    cell_lo: float = 0.0
    cell_hi: float = 1.0
    counts: object = None          # int32 [2] or None

    def c(self) -> _CSurrogate:
        torch = _torch()
        f32 = torch.float32
        lin = _arg(self.lin, "surrogate.lin", f32, (None, None))
        n_out, n_in = (int(x) for x in self.lin.shape)
        P = 64 * n_in + 64 + 64 * 64 + 64 + n_out * 64 + n_out
        return _CSurrogate(n_in, n_out, _arg(self.params, "surrogate.params", f32, (P,)),
                           _arg(self.in_scale, "surrogate.in_scale", f32, (n_in,)),
                           _arg(self.out_scale, "surrogate.out_scale", f32, (n_out,)), lin,
                           _arg(self.cell_ok, "surrogate.cell_ok", torch.uint8, (n_in * 16,), optional=True),
                           float(self.cell_lo), float(self.cell_hi),
                           _arg(self.counts, "surrogate.counts", torch.int32, (2,), optional=True))


@dataclass
class MlpTrain:
    """Adam state of surrogate training (device tensors); step counts updates done."""
    params: object
    adam_m: object
    adam_v: object
    step: int = 0
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self) -> _CTrain:
        f32 = _torch().float32
        p = _arg(self.params, "train.params", f32, (None,))
        n = (int(self.params.numel()),)
        return _CTrain(p, _arg(self.adam_m, "train.adam_m", f32, n), _arg(self.adam_v, "train.adam_v", f32, n),
                       int(self.step), float(self.lr), float(self.beta1), float(self.beta2), float(self.eps))


@dataclass
class Problem:
    geometry: Geometry
    phantom: Phantom
    spectral: Spectral
    scatter: Optional[Scatter] = None
    psf: Optional[Psf] = None


def _problem_c(pb: Problem):
    """C descriptors of a problem after the cross-checks between its tensors:
    scatter maps [A][nv][nu], per-bin scales [E], flood [nv][nu], one spread
    kernel per group.  Returns (geometry, phantom, spectral, keep, scatter, psf);
    keep holds host memory the spectral descriptor points to."""
    g = pb.geometry
    cg, cp = g.c(), pb.phantom.c()
    cs, keep = pb.spectral.c()
    E = int(pb.spectral.mu.shape[1])
    if pb.spectral.flood is not None and tuple(pb.spectral.flood.shape) != (g.nv, g.nu):
        raise ValueError(f"spectral.flood must have shape [{g.nv}][{g.nu}], not {list(pb.spectral.flood.shape)}")
    sc = ps = None
    if pb.scatter is not None:
        sc = pb.scatter.c()
        if tuple(pb.scatter.maps.shape) != (g.n_angles, g.nv, g.nu):
            raise ValueError(f"scatter.maps must have shape [{g.n_angles}][{g.nv}][{g.nu}], "
                             f"not {list(pb.scatter.maps.shape)}")
        if pb.scatter.s_bin is not None and int(pb.scatter.s_bin.numel()) != E:
            raise ValueError(f"scatter.s_bin must have {E} entries")
    if pb.psf is not None:
        ps = pb.psf.c()
        if int(pb.psf.kernels.shape[0]) != pb.spectral.n_groups:
            raise ValueError(f"psf.kernels must hold one kernel per group ({pb.spectral.n_groups}), "
                             f"not {int(pb.psf.kernels.shape[0])}")
    return cg, cp, cs, keep, sc, ps


def _ref(x):
    return C.byref(x) if x is not None else None


@_entry
def upload(cfg, device="cuda", scatter: bool = True, psf: bool = True) -> Problem:
    """Copy a host problem (attributes as in the ``synth`` configurations) to the GPU."""
    torch = _require_gpu()
    g, p, s = cfg.geometry, cfg.phantom, cfg.spectral
    dev = torch.device(device)
    ang = None if g.angles is None else torch.as_tensor(np.asarray(g.angles, np.float64), device=dev)
    geo = Geometry(float(g.sid), float(g.sdd), int(g.nu), int(g.nv), float(g.du), float(g.dv),
                   int(g.n_angles), float(g.off_u), float(g.off_v), ang)
    ph = Phantom(torch.as_tensor(np.ascontiguousarray(p.labels, dtype=np.int8), device=dev),
                 float(p.dx), float(p.dy), float(p.dz), float(p.cx), float(p.cy), float(p.cz))
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
    sp = Spectral(f32(s.mu), f32(s.phi), f32(s.eta), int(s.n_groups),
                  None if s.group_of_bin is None else np.asarray(s.group_of_bin, np.int32),
                  None if s.flood is None else f32(s.flood))
    sc = None
    if scatter and getattr(cfg, "scatter", None) is not None:
        sc = Scatter(f32(cfg.scatter.maps()), None if cfg.scatter.s_bin is None else f32(cfg.scatter.s_bin))
    ps = None
    if psf and getattr(cfg, "psf", None) is not None:
        ps = Psf(f32(cfg.psf.kernels))
    return Problem(geo, ph, sp, sc, ps)


# ------------------------------------------------------------ entry points

def fcat_version() -> int:
    return int(load().fcat_version())


def fcat_status_string(status: int) -> str:
    return load().fcat_status_string(int(status)).decode()


def fcat_last_error() -> str:
    return load().fcat_last_error().decode()


@_entry
def fcat_project_workspace_bytes(pb: Problem, mode: str = "plain", angles_per_chunk: int = 0) -> int:
    g, p, cs, _keep, sc, ps = _problem_c(pb)
    return int(load().fcat_project_workspace_bytes(C.byref(g), C.byref(p), C.byref(cs), _ref(sc), _ref(ps),
                                                   _mode(mode), int(angles_per_chunk)))


def _mode(mode: str) -> int:
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}, not {mode!r}")
    return MODES[mode]


def _workspace(nbytes: int, device):
    torch = _torch()
    if nbytes <= 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


@_entry
def fcat_project(pb: Problem, mode: str = "plain", surrogate=None, out=None, workspace=None,
                 angles_per_chunk: int = 0, stream=None, check: bool = False):
    """out[a][v][u] for all angles; allocates ``out`` and the workspace if not given.

    With ``check`` the call then waits for the stream and raises FcatError
    (FCAT_E_LABEL_RANGE / FCAT_E_NONFINITE) for the input problems the
    kernels noted (fcat_project_status); without it nothing synchronises."""
    g = pb.geometry
    cg, cp, cs, _keep, sc, ps = _problem_c(pb)
    md = _mode(mode)
    su = surrogate.c() if surrogate is not None else None
    if out is not None:
        _arg(out, "out", _torch().float32, (g.n_angles, g.nv, g.nu))
    _ws(workspace)
    torch = _require_gpu()
    lib = load()
    dev = pb.phantom.labels.device
    if out is None:
        out = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_project_workspace_bytes(pb, mode, angles_per_chunk), dev)
    wp, wn = _ws(workspace)
    st = lib.fcat_project(C.byref(cg), C.byref(cp), C.byref(cs), _ref(sc), _ref(ps), md, _ref(su),
                          _ptr(out), wp, wn, _stream(stream))
    _check(st)
    if check:
        fcat_project_status(workspace, stream)
    return out


@_entry
def fcat_project_status(workspace, stream=None) -> None:
    """Raises FcatError(FCAT_E_LABEL_RANGE / FCAT_E_NONFINITE) for the input
    problems that the last fcat_project / fcat_projections call with this
    workspace noted; waits for the stream."""
    wp, wn = _ws(workspace)
    _require_gpu()
    _check(load().fcat_project_status(wp, wn, _stream(stream)))


@_entry
def project(geometry: Geometry, labels, mu, phi, eta, scatter=None, psf=None, mode: str = "plain", *,
            voxel=None, centre=(0.0, 0.0, 0.0), group_of_bin=None, flood=None, surrogate=None, stream=None,
            check: bool = True):
    """Projections [A][nv][nu] of one phantom from plain device tensors (marshalling only).

    labels: a Phantom, or a device int8 tensor [nz][ny][nx] with voxel = (dx, dy, dz)
    in mm and the volume centre ``centre``; mu [M][E], phi [E], eta [E] device
    float32; scatter: None, a Scatter or a device float32 [A][nv][nu]; psf:
    None, a Psf or a device float32 [G][k][k].  The number of energy groups is
    G of the PSF (the groups of ``group_of_bin``, else an even split of the
    bins); without a PSF it is the number of groups of ``group_of_bin``, else 1.
    With ``check`` (the default) labels outside 0..M-1 and non-finite inputs
    raise FcatError after the call (it then waits for the stream).
    """
    if isinstance(labels, Phantom):
        ph = labels
    else:
        if voxel is None:
            raise ValueError("project: voxel=(dx, dy, dz) is required with a labels tensor")
        ph = Phantom(labels, *(float(v) for v in voxel), *(float(c) for c in centre))
    sc = scatter if scatter is None or isinstance(scatter, Scatter) else Scatter(scatter)
    ps = psf if psf is None or isinstance(psf, Psf) else Psf(psf)
    if ps is not None:
        n_groups = int(ps.kernels.shape[0])
    elif group_of_bin is not None:
        n_groups = int(np.max(np.asarray(group_of_bin))) + 1
    else:
        n_groups = 1
    sp = Spectral(mu, phi, eta, n_groups, None if group_of_bin is None else np.asarray(group_of_bin, np.int32), flood)
    return fcat_project(Problem(geometry, ph, sp, sc, ps), mode=mode, surrogate=surrogate, stream=stream,
                        check=check)


@_entry
def fcat_pathlengths_workspace_bytes(phantom: Phantom) -> int:
    cp = phantom.c()
    return int(load().fcat_pathlengths_workspace_bytes(C.byref(cp)))


@_entry
def fcat_pathlengths(pb: Problem, n_mat: int, a_begin: int = 0, a_end: Optional[int] = None,
                     out=None, workspace=None, stream=None):
    """L[a][v][u][m] for angles a_begin <= a < a_end."""
    g = pb.geometry
    a_end = g.n_angles if a_end is None else a_end
    cg, cp = g.c(), pb.phantom.c()
    if out is not None:
        _arg(out, "out", _torch().float32, (max(a_end - a_begin, 0), g.nv, g.nu, n_mat))
    _ws(workspace)
    torch = _require_gpu()
    dev = pb.phantom.labels.device
    if out is None:
        out = torch.empty((max(a_end - a_begin, 0), g.nv, g.nu, n_mat), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_pathlengths_workspace_bytes(pb.phantom), dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_pathlengths(C.byref(cg), C.byref(cp), int(n_mat), int(a_begin), int(a_end),
                                   _ptr(out), wp, wn, _stream(stream)))
    return out


WALK_COUNTS = ("hit_rays", "brick_steps", "mixed_bricks", "voxel_steps", "voxel_lane_slots", "siddon_segments")


@_entry
def fcat_walk_stats(pb: Problem, a_begin: int = 0, a_end: Optional[int] = None, workspace=None,
                    stream=None) -> dict:
    """Step counts of the exact walk over angles a_begin <= a < a_end (synchronises)."""
    g = pb.geometry
    a_end = g.n_angles if a_end is None else a_end
    cg, cp = g.c(), pb.phantom.c()
    _ws(workspace)
    torch = _require_gpu()
    dev = pb.phantom.labels.device
    counts = torch.empty(len(WALK_COUNTS), dtype=torch.int64, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_pathlengths_workspace_bytes(pb.phantom), dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_walk_stats(C.byref(cg), C.byref(cp), int(a_begin), int(a_end), _ptr(counts), wp, wn,
                                  _stream(stream)))
    return dict(zip(WALK_COUNTS, (int(x) for x in counts.cpu().tolist())))


@_entry
def fcat_spectral_workspace_bytes(spectral: Spectral) -> int:
    cs, _keep = spectral.c()
    return int(load().fcat_spectral_workspace_bytes(C.byref(cs)))


@_entry
def fcat_spectral(L, spectral: Spectral, i0=None, S=None, s_bin=None, mode: str = "plain", out=None,
                  workspace=None, stream=None):
    """Y[g][r] from L[r][m] (Eq. 3 per ray)."""
    f32 = _torch().float32
    cs, _keep = spectral.c()
    M, E = (int(x) for x in spectral.mu.shape)
    pL = _arg(L, "L", f32, (None, M))
    n = int(L.shape[0])
    pi0 = _arg(i0, "i0", f32, (n,), optional=True)
    pS = _arg(S, "S", f32, (n,), optional=True)
    psb = _arg(s_bin, "s_bin", f32, (E,), optional=True)
    if out is not None:
        _arg(out, "out", f32, (spectral.n_groups, n))
    md = _mode(mode)
    _ws(workspace)
    torch = _require_gpu()
    if out is None:
        out = torch.empty((spectral.n_groups, n), dtype=torch.float32, device=L.device)
    if workspace is None:
        workspace = _workspace(fcat_spectral_workspace_bytes(spectral), L.device)
    wp, wn = _ws(workspace)
    _check(load().fcat_spectral(pL, n, C.byref(cs), pi0, pS, psb, md, _ptr(out), wp, wn, _stream(stream)))
    return out


@_entry
def fcat_spectral_static(L, spectral: Spectral, i0=None, S=None, s_bin=None, mode: str = "plain", out=None,
                         stream=None):
    """fcat_spectral with its tables in the library's static scratch (no workspace)."""
    f32 = _torch().float32
    cs, _keep = spectral.c()
    M, E = (int(x) for x in spectral.mu.shape)
    pL = _arg(L, "L", f32, (None, M))
    n = int(L.shape[0])
    pi0 = _arg(i0, "i0", f32, (n,), optional=True)
    pS = _arg(S, "S", f32, (n,), optional=True)
    psb = _arg(s_bin, "s_bin", f32, (E,), optional=True)
    if out is not None:
        _arg(out, "out", f32, (spectral.n_groups, n))
    md = _mode(mode)
    torch = _require_gpu()
    if out is None:
        out = torch.empty((spectral.n_groups, n), dtype=torch.float32, device=L.device)
    _check(load().fcat_spectral_static(pL, n, C.byref(cs), pi0, pS, psb, md, _ptr(out), _stream(stream)))
    return out


@_entry
def fcat_psf(Y, psf: Psf, out=None, stream=None):
    """out[a][v][u] = sum_g K_g (*) Y[a][g] for Y[a][g][v][u]."""
    f32 = _torch().float32
    pY = _arg(Y, "Y", f32, (None, None, None, None))
    A, G, nv, nu = (int(x) for x in Y.shape)
    cps = psf.c()
    if int(psf.kernels.shape[0]) != G:
        raise ValueError(f"psf.kernels must hold one kernel per group of Y ({G})")
    if out is not None:
        _arg(out, "out", f32, (A, nv, nu))
    torch = _require_gpu()
    if out is None:
        out = torch.empty((A, nv, nu), dtype=torch.float32, device=Y.device)
    _check(load().fcat_psf(pY, A, G, nv, nu, C.byref(cps), _ptr(out), _stream(stream)))
    return out


@_entry
def fcat_check_inputs(pb: Problem, workspace=None, stream=None) -> None:
    """Raises FcatError(FCAT_E_LABEL_RANGE / FCAT_E_NONFINITE) on bad device data."""
    cg, cp, cs, _keep, sc, ps = _problem_c(pb)
    _ws(workspace)
    _require_gpu()
    dev = pb.phantom.labels.device
    if workspace is None:
        workspace = _workspace(256, dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_check_inputs(C.byref(cg), C.byref(cp), C.byref(cs), _ref(sc), _ref(ps), wp, wn,
                                    _stream(stream)))


@_entry
def fcat_timing_enable(enable: bool = True) -> None:
    """Bracket every library kernel launch with HIP events (process-wide)."""
    _check(load().fcat_timing_enable(1 if enable else 0))


@_entry
def fcat_timing_read(reset: bool = True) -> dict:
    """{stage: (total_ms, launches)} of the launches recorded since the last reset."""
    n = len(STAGES)
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(load().fcat_timing_read(ms, cnt, n, 1 if reset else 0))
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


# ------------------------------------------------- noise and projections

@dataclass
class Noise:
    """Eq. 5 noise: H = counts_per_pixel flood counts per open pixel."""
    counts_per_pixel: float
    seed: int = 0
    floor: float = 0.0

    def c(self) -> _CNoise:
        return _CNoise(float(self.counts_per_pixel), int(self.seed) & 0xFFFFFFFFFFFFFFFF, float(self.floor))


@_entry
def fcat_count_scale(spectral: Spectral, counts_per_pixel: float, out=None, stream=None):
    """c_g = H Phi_g / (Phi W_g) as a device float tensor [G]."""
    cs, _keep = spectral.c()
    if out is not None:
        _arg(out, "out", _torch().float32, (spectral.n_groups,))
    torch = _require_gpu()
    if out is None:
        out = torch.empty(spectral.n_groups, dtype=torch.float32, device=spectral.mu.device)
    _check(load().fcat_count_scale(C.byref(cs), float(counts_per_pixel), _ptr(out), _stream(stream)))
    return out


@_entry
def fcat_poisson(Y, scale, seed: int, angle_base: int = 0, stream=None):
    """In place: Y[a][g][...] <- Poisson(scale[g] Y) / scale[g] for float32 Y [A][G][plane...]."""
    f32 = _torch().float32
    if Y is None or getattr(Y, "dim", lambda: 0)() < 3:
        raise ValueError("Y must be a float32 tensor [A][G][plane...]")
    pY = _arg(Y, "Y", f32, tuple([None] * Y.dim()))
    A, G = int(Y.shape[0]), int(Y.shape[1])
    plane = int(math.prod(Y.shape[2:]))
    ps = _arg(scale, "scale", f32, (G,))
    _require_gpu()
    _check(load().fcat_poisson(pY, A, G, plane, ps, int(seed) & 0xFFFFFFFFFFFFFFFF, int(angle_base),
                               _stream(stream)))
    return Y


@_entry
def fcat_flood_workspace_bytes(spectral: Spectral, nv: int, nu: int) -> int:
    cs, _keep = spectral.c()
    return int(load().fcat_flood_workspace_bytes(C.byref(cs), int(nv), int(nu)))


@_entry
def fcat_flood_profile(spectral: Spectral, psf: Optional[Psf], nv: int, nu: int, out=None, workspace=None,
                       stream=None):
    """Noiseless object-free flood through the spread, [nv][nu]."""
    cs, _keep = spectral.c()
    ps = psf.c() if psf is not None else None
    if out is not None:
        _arg(out, "out", _torch().float32, (nv, nu))
    _ws(workspace)
    torch = _require_gpu()
    dev = spectral.mu.device
    if out is None:
        out = torch.empty((nv, nu), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_flood_workspace_bytes(spectral, nv, nu), dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_flood_profile(C.byref(cs), _ref(ps), int(nv), int(nu), _ptr(out), wp, wn, _stream(stream)))
    return out


@_entry
def fcat_log_projection(out, flood, floor: float = 0.0, proj=None, stream=None):
    """-ln(max(out, floor) / flood) for out [A][plane...], flood [plane...]."""
    f32 = _torch().float32
    if out is None or getattr(out, "dim", lambda: 0)() < 2:
        raise ValueError("out must be a float32 tensor [A][plane...]")
    po = _arg(out, "out", f32, tuple([None] * out.dim()))
    pf = _arg(flood, "flood", f32, tuple(int(x) for x in out.shape[1:]))
    A = int(out.shape[0])
    plane = int(flood.numel())
    if proj is not None:
        _arg(proj, "proj", f32, tuple(int(x) for x in out.shape))
    torch = _require_gpu()
    if proj is None:
        proj = torch.empty_like(out)
    _check(load().fcat_log_projection(po, pf, A, plane, float(floor), _ptr(proj), _stream(stream)))
    return proj


@_entry
def fcat_projections_workspace_bytes(pb: Problem, mode: str = "plain", angles_per_chunk: int = 0) -> int:
    g, p, cs, _keep, sc, ps = _problem_c(pb)
    return int(load().fcat_projections_workspace_bytes(C.byref(g), C.byref(p), C.byref(cs), _ref(sc), _ref(ps),
                                                       _mode(mode), int(angles_per_chunk)))


@_entry
def fcat_projections(pb: Problem, noise: Optional[Noise] = None, mode: str = "plain", surrogate=None, out=None,
                     workspace=None, angles_per_chunk: int = 0, stream=None):
    """Projections -ln(out / flood) of all angles, with Poisson noise when ``noise`` is given."""
    g = pb.geometry
    cg, cp, cs, _keep, sc, ps = _problem_c(pb)
    md = _mode(mode)
    su = surrogate.c() if surrogate is not None else None
    nz = noise.c() if noise is not None else None
    if out is not None:
        _arg(out, "out", _torch().float32, (g.n_angles, g.nv, g.nu))
    _ws(workspace)
    torch = _require_gpu()
    lib = load()
    dev = pb.phantom.labels.device
    if out is None:
        out = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_projections_workspace_bytes(pb, mode, angles_per_chunk), dev)
    wp, wn = _ws(workspace)
    st = lib.fcat_projections(C.byref(cg), C.byref(cp), C.byref(cs), _ref(sc), _ref(ps), md, _ref(su), _ref(nz),
                              _ptr(out), wp, wn, _stream(stream))
    _check(st)
    return out


# ------------------------------------------------------------------ dose

@_entry
def fcat_dose_workspace_bytes(pb: Problem, angles_per_chunk: int = 0) -> int:
    cs, _keep = pb.spectral.c()
    g, p = pb.geometry.c(), pb.phantom.c()
    return int(load().fcat_dose_workspace_bytes(C.byref(g), C.byref(p), C.byref(cs), int(angles_per_chunk)))


@_entry
def fcat_dose(pb: Problem, energy, mu_en_over_mu, mass: float, a_begin: int = 0, a_end: Optional[int] = None,
              workspace=None, angles_per_chunk: int = 0, stream=None):
    """(D0 [E] float64 device tensor, Dp [1]) of Eqs. 6-7 over angles a_begin <= a < a_end."""
    g = pb.geometry
    a_end = g.n_angles if a_end is None else a_end
    cs, _keep = pb.spectral.c()
    cg, cp = g.c(), pb.phantom.c()
    E = int(pb.spectral.mu.shape[1])
    f32 = _torch().float32
    pe = _arg(energy, "energy", f32, (E,))
    pr = _arg(mu_en_over_mu, "mu_en_over_mu", f32, (E,))
    _ws(workspace)
    torch = _require_gpu()
    dev = pb.phantom.labels.device
    D0 = torch.empty(E, dtype=torch.float64, device=dev)
    Dp = torch.empty(1, dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_dose_workspace_bytes(pb, angles_per_chunk), dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_dose(C.byref(cg), C.byref(cp), C.byref(cs), pe, pr, float(mass), int(a_begin), int(a_end),
                            _ptr(D0), _ptr(Dp), wp, wn, _stream(stream)))
    return D0, Dp


# ------------------------------------------------------------- reconstruction

def _cgrid(grid) -> _CGrid:
    return _CGrid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.dx), float(grid.dy), float(grid.dz),
                  float(grid.cx), float(grid.cy), float(grid.cz))


def _proj_arg(t, name: str, geometry: Geometry, n=None) -> int:
    """A stack of detector images [n][nv][nu] of the geometry."""
    return _arg(t, name, _torch().float32, (n, geometry.nv, geometry.nu))


@_entry
def fcat_fdk_filter(geometry: Geometry, proj, out=None, stream=None):
    """Cosine-weighted, ramp-filtered projections [n_ang][nv][nu]."""
    cg = geometry.c()
    pp = _proj_arg(proj, "proj", geometry)
    if out is not None:
        _proj_arg(out, "out", geometry, int(proj.shape[0]))
    torch = _require_gpu()
    if out is None:
        out = torch.empty_like(proj)
    _check(load().fcat_fdk_filter(C.byref(cg), pp, int(proj.shape[0]), _ptr(out), _stream(stream)))
    return out


@_entry
def fcat_fdk_backproject_workspace_bytes(n_ang: int) -> int:
    return int(load().fcat_fdk_backproject_workspace_bytes(int(n_ang)))


@_entry
def fcat_fdk_backproject(geometry: Geometry, filtered, grid, a_begin: int = 0, volume=None, accumulate: bool = False,
                         workspace=None, stream=None):
    """FDK back-projection of filtered projections of angles a_begin .. a_begin + n - 1."""
    cg, cv = geometry.c(), _cgrid(grid)
    pf = _proj_arg(filtered, "filtered", geometry)
    n = int(filtered.shape[0])
    if volume is not None:
        _arg(volume, "volume", _torch().float32, (grid.nz, grid.ny, grid.nx))
    _ws(workspace)
    torch = _require_gpu()
    if volume is None:
        volume = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float32, device=filtered.device)
    if workspace is None:
        workspace = _workspace(fcat_fdk_backproject_workspace_bytes(n), filtered.device)
    wp, wn = _ws(workspace)
    _check(load().fcat_fdk_backproject(C.byref(cg), pf, int(a_begin), int(a_begin) + n, C.byref(cv),
                                       _ptr(volume), 1 if accumulate else 0, wp, wn, _stream(stream)))
    return volume


@_entry
def fcat_fdk_workspace_bytes(geometry: Geometry, angles_per_chunk: int = 0) -> int:
    cg = geometry.c()
    return int(load().fcat_fdk_workspace_bytes(C.byref(cg), int(angles_per_chunk)))


@_entry
def fcat_fdk(geometry: Geometry, proj, grid, volume=None, workspace=None, angles_per_chunk: int = 0, stream=None):
    """FDK reconstruction [nz][ny][nx] (mm^-1) of projections [n_angles][nv][nu]."""
    cg, cv = geometry.c(), _cgrid(grid)
    pp = _proj_arg(proj, "proj", geometry, geometry.n_angles)
    if volume is not None:
        _arg(volume, "volume", _torch().float32, (grid.nz, grid.ny, grid.nx))
    _ws(workspace)
    torch = _require_gpu()
    if volume is None:
        volume = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float32, device=proj.device)
    if workspace is None:
        workspace = _workspace(fcat_fdk_workspace_bytes(geometry, angles_per_chunk), proj.device)
    wp, wn = _ws(workspace)
    _check(load().fcat_fdk(C.byref(cg), pp, C.byref(cv), _ptr(volume), wp, wn, _stream(stream)))
    return volume


# ------------------------------------------------------- image projector pair

@_entry
def fcat_image_project(geometry: Geometry, grid, image, a_begin: int = 0, a_end: Optional[int] = None, out=None,
                       stream=None):
    """(A f)[a][v][u]: line integrals of image [nz][ny][nx] for angles a_begin <= a < a_end."""
    a_end = geometry.n_angles if a_end is None else a_end
    cg, cv = geometry.c(), _cgrid(grid)
    f32 = _torch().float32
    pi = _arg(image, "image", f32, (grid.nz, grid.ny, grid.nx))
    if out is not None:
        _arg(out, "out", f32, (a_end - a_begin, geometry.nv, geometry.nu))
    torch = _require_gpu()
    if out is None:
        out = torch.empty((a_end - a_begin, geometry.nv, geometry.nu), dtype=torch.float32, device=image.device)
    _check(load().fcat_image_project(C.byref(cg), C.byref(cv), pi, int(a_begin), int(a_end), _ptr(out),
                                     _stream(stream)))
    return out


@_entry
def fcat_image_backproject(geometry: Geometry, grid, proj, a_begin: int = 0, image=None, accumulate: bool = False,
                           stream=None):
    """(A^T y)[nz][ny][nx] for y = proj [n][nv][nu] of angles a_begin .. a_begin + n - 1."""
    cg, cv = geometry.c(), _cgrid(grid)
    f32 = _torch().float32
    pp = _arg(proj, "proj", f32, (None, geometry.nv, geometry.nu))
    n = int(proj.shape[0])
    if image is not None:
        _arg(image, "image", f32, (grid.nz, grid.ny, grid.nx))
    torch = _require_gpu()
    if image is None:
        image = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float32, device=proj.device)
    _check(load().fcat_image_backproject(C.byref(cg), C.byref(cv), pp, int(a_begin), int(a_begin) + n,
                                         _ptr(image), 1 if accumulate else 0, _stream(stream)))
    return image


# ------------------------------------------------------------- detector optics

@_entry
def fcat_effective_psf(spectral: Spectral, psf: Psf, out=None, stream=None):
    """sum_g W_g K_g / sum_g W_g as a device float tensor [k][k]."""
    cs, _keep = spectral.c()
    cps = psf.c()
    k = int(psf.kernels.shape[1])
    if out is not None:
        _arg(out, "out", _torch().float32, (k, k))
    torch = _require_gpu()
    if out is None:
        out = torch.empty((k, k), dtype=torch.float32, device=psf.kernels.device)
    _check(load().fcat_effective_psf(C.byref(cs), C.byref(cps), _ptr(out), _stream(stream)))
    return out


@_entry
def fcat_slit_lsf_range(pitch: float, tilt_deg: float, n_rows: int, n_cols: int, oversample: int):
    """(b_min, n_bins) of the presampled LSF."""
    b, n = C.c_int32(), C.c_int32()
    _check(load().fcat_slit_lsf_range(float(pitch), float(tilt_deg), int(n_rows), int(n_cols), int(oversample),
                                      C.byref(b), C.byref(n)))
    return int(b.value), int(n.value)


@_entry
def fcat_slit_mtf(kernel, pitch: float, width: float, tilt_deg: float, n_rows: int, n_cols: int, oversample: int,
                  freqs, stream=None):
    """(mtf [n_freq], lsf [n_bins], counts [n_bins], b_min) as device tensors (float64, int32)."""
    pk = _arg(kernel, "kernel", _torch().float32, (None, None))
    k = int(kernel.shape[0])
    if int(kernel.shape[1]) != k:
        raise ValueError(f"kernel must be square, not {list(kernel.shape)}")
    torch = _require_gpu()
    dev = kernel.device
    b_min, n_bins = fcat_slit_lsf_range(pitch, tilt_deg, n_rows, n_cols, oversample)
    f = torch.as_tensor(np.asarray(freqs, np.float64), device=dev)
    mtf = torch.empty(f.numel(), dtype=torch.float64, device=dev)
    lsf = torch.empty(n_bins, dtype=torch.float64, device=dev)
    cnt = torch.empty(n_bins, dtype=torch.int32, device=dev)
    ws = _workspace(fcat_slit_mtf_workspace_bytes(n_rows, n_cols, n_bins), dev)
    wp, wn = _ws(ws)
    _check(load().fcat_slit_mtf(pk, k, float(pitch), float(width), float(tilt_deg), int(n_rows), int(n_cols),
                                int(oversample), _ptr(f), int(f.numel()), _ptr(mtf), _ptr(lsf), _ptr(cnt), wp, wn,
                                _stream(stream)))
    return mtf, lsf, cnt, b_min


@_entry
def fcat_richardson_lucy_workspace_bytes(n: int, nv: int, nu: int, k: int) -> int:
    return int(load().fcat_richardson_lucy_workspace_bytes(int(n), int(nv), int(nu), int(k)))


@_entry
def fcat_slit_mtf_workspace_bytes(n_rows: int, n_cols: int, n_bins: int) -> int:
    return int(load().fcat_slit_mtf_workspace_bytes(int(n_rows), int(n_cols), int(n_bins)))


@_entry
def fcat_richardson_lucy(images, kernel, iterations: int, out=None, workspace=None, stream=None):
    """Richardson-Lucy deconvolution of images [n][nv][nu] with one kernel [k][k]."""
    f32 = _torch().float32
    pi = _arg(images, "images", f32, (None, None, None))
    n, nv, nu = (int(x) for x in images.shape)
    pk = _arg(kernel, "kernel", f32, (None, None))
    k = int(kernel.shape[0])
    if int(kernel.shape[1]) != k:
        raise ValueError(f"kernel must be square, not {list(kernel.shape)}")
    if out is not None:
        _arg(out, "out", f32, (n, nv, nu))
    _ws(workspace)
    torch = _require_gpu()
    if out is None:
        out = torch.empty_like(images)
    if workspace is None:
        workspace = _workspace(fcat_richardson_lucy_workspace_bytes(n, nv, nu, k), images.device)
    wp, wn = _ws(workspace)
    _check(load().fcat_richardson_lucy(pi, n, nv, nu, pk, k, int(iterations), _ptr(out), wp, wn, _stream(stream)))
    return out


# ------------------------------------------------------------- surrogate

@_entry
def fcat_mlp_param_count(n_in: int, n_out: int) -> int:
    return int(load().fcat_mlp_param_count(int(n_in), int(n_out)))


@_entry
def fcat_mlp_workspace_bytes(spectral: Spectral, batch: int) -> int:
    cs, _keep = spectral.c()
    return int(load().fcat_mlp_workspace_bytes(C.byref(cs), int(batch)))


def _mlp_ws(spectral: Spectral, batch: int, device, workspace):
    if workspace is not None:
        _ws(workspace)
        return workspace
    return _workspace(fcat_mlp_workspace_bytes(spectral, batch), device)


def _samples(spectral: Spectral, L, Yprim=None):
    """Pointers of a sample set: L [n][M], Yprim [G][n] (float32, device)."""
    f32 = _torch().float32
    M = int(spectral.mu.shape[0])
    pL = _arg(L, "L", f32, (None, M))
    n = int(L.shape[0])
    pY = _arg(Yprim, "Yprim", f32, (spectral.n_groups, n)) if Yprim is not None else None
    return pL, pY, n


@_entry
def fcat_mlp_linear_term(spectral: Spectral, out=None, workspace=None, stream=None):
    """lin[g][m] = sum_{e in g} w_e mu[m][e] / W_g."""
    cs, _keep = spectral.c()
    M, _E = (int(x) for x in spectral.mu.shape)
    if out is not None:
        _arg(out, "out", _torch().float32, (spectral.n_groups, M))
    _ws(workspace)
    torch = _require_gpu()
    dev = spectral.mu.device
    if out is None:
        out = torch.empty((spectral.n_groups, M), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(fcat_spectral_workspace_bytes(spectral), dev)
    wp, wn = _ws(workspace)
    _check(load().fcat_mlp_linear_term(C.byref(cs), _ptr(out), wp, wn, _stream(stream)))
    return out


@_entry
def fcat_mlp_forward(sur: Surrogate, spectral: Spectral, L, out=None, workspace=None, stream=None):
    """Network prediction of Yprim[g][r] for L[r][m] (no fallback)."""
    cs, _keep = spectral.c()
    cu = sur.c()
    pL, _, n = _samples(spectral, L)
    if out is not None:
        _arg(out, "out", _torch().float32, (spectral.n_groups, n))
    torch = _require_gpu()
    if out is None:
        out = torch.empty((spectral.n_groups, n), dtype=torch.float32, device=L.device)
    ws = _mlp_ws(spectral, 1, L.device, workspace)
    wp, wn = _ws(ws)
    _check(load().fcat_mlp_forward(C.byref(cu), C.byref(cs), pL, n, _ptr(out), wp, wn, _stream(stream)))
    return out


@_entry
def fcat_mlp_gradients(sur: Surrogate, spectral: Spectral, L, Yprim, workspace=None, stream=None):
    """(loss, grad) of the mean squared residual error over all samples."""
    cs, _keep = spectral.c()
    cu = sur.c()
    pL, pY, n = _samples(spectral, L, Yprim)
    torch = _require_gpu()
    grad = torch.empty_like(sur.params)
    loss = torch.empty(1, dtype=torch.float32, device=L.device)
    ws = _mlp_ws(spectral, n, L.device, workspace)
    wp, wn = _ws(ws)
    _check(load().fcat_mlp_gradients(C.byref(cu), C.byref(cs), pL, pY, n, _ptr(grad), _ptr(loss), wp, wn,
                                     _stream(stream)))
    return loss, grad


@_entry
def fcat_mlp_train_step(train: MlpTrain, sur: Surrogate, spectral: Spectral, L, Yprim, order=None, base: int = 0,
                        count: Optional[int] = None, loss=None, workspace=None, stream=None):
    """One Adam step on samples order[base:base+count] (or base:base+count)."""
    cs, _keep = spectral.c()
    cu, ct = sur.c(), train.c()
    pL, pY, n = _samples(spectral, L, Yprim)
    po = _arg(order, "order", _torch().int32, (None,), optional=True)
    pl = _arg(loss, "loss", _torch().float32, (1,), optional=True)
    count = n - base if count is None else count
    ws = _mlp_ws(spectral, count, L.device, workspace)
    wp, wn = _ws(ws)
    _require_gpu()
    _check(load().fcat_mlp_train_step(C.byref(ct), C.byref(cu), C.byref(cs), pL, pY, n, po, int(base), int(count),
                                      pl, wp, wn, _stream(stream)))
    train.step = int(ct.step)


@_entry
def fcat_mlp_train_epoch(train: MlpTrain, sur: Surrogate, spectral: Spectral, L, Yprim, order, batch: int,
                         batch_loss=None, workspace=None, stream=None):
    """Minibatch Adam steps over order[0:n]."""
    cs, _keep = spectral.c()
    cu, ct = sur.c(), train.c()
    pL, pY, n = _samples(spectral, L, Yprim)
    po = _arg(order, "order", _torch().int32, (n,))
    pbl = _arg(batch_loss, "batch_loss", _torch().float32, (None,), optional=True)
    ws = _mlp_ws(spectral, batch, L.device, workspace)
    wp, wn = _ws(ws)
    _require_gpu()
    _check(load().fcat_mlp_train_epoch(C.byref(ct), C.byref(cu), C.byref(cs), pL, pY, n, po, int(batch), pbl, wp,
                                       wn, _stream(stream)))
    train.step = int(ct.step)


@_entry
def fcat_mlp_validate(sur: Surrogate, spectral: Spectral, L, Yprim, threshold: float = 1e-3, min_count: int = 8,
                      workspace=None, stream=None):
    """(cell_err, cell_ok, cell_count) of the held-out set; also stores cell_ok in ``sur``."""
    cs, _keep = spectral.c()
    cu = sur.c()
    pL, pY, n = _samples(spectral, L, Yprim)
    torch = _require_gpu()
    n_out, n_in = (int(x) for x in sur.lin.shape)
    dev = L.device
    cell_err = torch.empty(n_in * 16, dtype=torch.float32, device=dev)
    cell_ok = torch.empty(n_in * 16, dtype=torch.uint8, device=dev)
    cell_count = torch.empty(n_in * 16, dtype=torch.int32, device=dev)
    ws = _mlp_ws(spectral, 1, dev, workspace)
    wp, wn = _ws(ws)
    _check(load().fcat_mlp_validate(C.byref(cu), C.byref(cs), pL, pY, n, float(threshold), int(min_count),
                                    _ptr(cell_err), _ptr(cell_ok), _ptr(cell_count), wp, wn, _stream(stream)))
    sur.cell_ok = cell_ok
    return cell_err, cell_ok, cell_count


@_entry
def fcat_mlp_setup(spectral: Spectral, lin, L, Yprim, workspace=None, stream=None):
    """(in_scale, out_scale, tau_max) of a training set (device tensors)."""
    cs, _keep = spectral.c()
    M = int(spectral.mu.shape[0])
    plin = _arg(lin, "lin", _torch().float32, (spectral.n_groups, M))
    pL, pY, n = _samples(spectral, L, Yprim)
    torch = _require_gpu()
    dev = L.device
    in_scale = torch.empty(M, dtype=torch.float32, device=dev)
    out_scale = torch.empty(spectral.n_groups, dtype=torch.float32, device=dev)
    tau_max = torch.empty(1, dtype=torch.float32, device=dev)
    ws = _mlp_ws(spectral, 1, dev, workspace)
    wp, wn = _ws(ws)
    _check(load().fcat_mlp_setup(C.byref(cs), plin, pL, pY, n, _ptr(in_scale), _ptr(out_scale), _ptr(tau_max),
                                 wp, wn, _stream(stream)))
    return in_scale, out_scale, tau_max
