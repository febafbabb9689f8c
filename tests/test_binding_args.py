"""Argument checks of the Python binding (CPU only, nothing reaches the GPU).

The C ABI takes raw pointers and cannot tell a host tensor, a float64 table,
a transposed view or a short output from the arrays it documents.  The
binding checks dtype, contiguity and shape of every caller tensor against
the descriptors, then that it lives on a GPU, and raises ValueError before
calling the library.  The checks run in that order, so each one can be
exercised here with host tensors.
"""
import numpy as np
import pytest
import torch

import paper_2011_04736_amd as fc

A, NV, NU, M, E, G, K = 3, 4, 16, 3, 5, 2, 5


def _problem(**over):
    f32 = torch.float32
    t = dict(
        labels=torch.zeros((4, 8, 8), dtype=torch.int8),
        mu=torch.ones((M, E), dtype=f32), phi=torch.ones(E, dtype=f32), eta=torch.ones(E, dtype=f32),
        flood=None, maps=torch.zeros((A, NV, NU), dtype=f32), s_bin=None,
        kernels=torch.ones((G, K, K), dtype=f32), angles=None,
    )
    t.update(over)
    geo = fc.Geometry(1000.0, 1500.0, NU, NV, 1.0, 1.0, A, angles=t["angles"])
    ph = fc.Phantom(t["labels"], 1.0, 1.0, 1.0)
    sp = fc.Spectral(t["mu"], t["phi"], t["eta"], G, flood=t["flood"])
    sc = fc.Scatter(t["maps"], t["s_bin"]) if t["maps"] is not None else None
    ps = fc.Psf(t["kernels"]) if t["kernels"] is not None else None
    return fc.Problem(geo, ph, sp, sc, ps)


def _raises(match, fn, *a, **k):
    with pytest.raises(ValueError, match=match):
        fn(*a, **k)


def test_well_formed_host_problem_is_refused_for_its_device():
    _raises("must be on a GPU", fc.fcat_project, _problem())
    _raises("must be on a GPU", fc.fcat_projections, _problem())
    _raises("must be on a GPU", fc.fcat_check_inputs, _problem())


@pytest.mark.parametrize("field,value,match", [
    ("mu", torch.ones((M, E), dtype=torch.float64), "spectral.mu must be torch.float32"),
    ("phi", torch.ones(E + 1), "spectral.phi must have shape"),
    ("eta", torch.ones((E, 1)), "spectral.eta must have shape"),
    ("labels", torch.zeros((8, 8, 4), dtype=torch.int8).transpose(0, 2), "phantom.labels must be contiguous"),
    ("labels", torch.zeros((4, 8, 8), dtype=torch.int32), "phantom.labels must be torch.int8"),
    ("labels", torch.zeros((32, 8), dtype=torch.int8), "phantom.labels must have shape"),
    ("maps", torch.zeros((A, NU, NV)), r"scatter.maps must have shape \[3\]\[4\]\[16\]"),
    ("maps", torch.zeros((A + 1, NV, NU)), "scatter.maps must have shape"),
    ("s_bin", torch.ones(E + 2), "scatter.s_bin must have 5 entries"),
    ("flood", torch.ones((NU, NV)), r"spectral.flood must have shape \[4\]\[16\]"),
    ("kernels", torch.ones((G + 1, K, K)), "one kernel per group"),
    ("kernels", torch.ones((G, K, K + 2)), r"psf.kernels must be \[G\]\[k\]\[k\]"),
    ("angles", torch.zeros(A, dtype=torch.float32), "geometry.angles must be torch.float64"),
    ("angles", torch.zeros(A + 1, dtype=torch.float64), "geometry.angles must have shape"),
])
def test_projector_descriptor_checks(field, value, match):
    pb = _problem(**{field: value})
    _raises(match, fc.fcat_project, pb)
    _raises(match, fc.fcat_projections, pb)


def test_projector_output_workspace_and_mode():
    pb = _problem()
    _raises(r"out must have shape \[3\]\[4\]\[16\]", fc.fcat_project, pb, out=torch.empty((A, NV, NU - 1)))
    _raises("out must be torch.float32", fc.fcat_project, pb, out=torch.empty((A, NV, NU), dtype=torch.float64))
    _raises("out must be contiguous", fc.fcat_project, pb, out=torch.empty((A, NU, NV)).transpose(1, 2))
    _raises("workspace must be a torch.Tensor", fc.fcat_project, pb, workspace=np.zeros(16, np.uint8))
    _raises("mode must be one of", fc.fcat_project, pb, mode="fp16")
    _raises("workspace must be on a GPU", fc.fcat_project_status, torch.zeros(256, dtype=torch.uint8))


def test_stage_entry_points():
    pb = _problem()
    sp = pb.spectral
    _raises(r"L must have shape \[\*\]\[3\]", fc.fcat_spectral, torch.zeros((10, M + 1)), sp)
    _raises("L must be torch.float32", fc.fcat_spectral, torch.zeros((10, M), dtype=torch.float64), sp)
    _raises(r"i0 must have shape \[10\]", fc.fcat_spectral, torch.zeros((10, M)), sp, i0=torch.ones(9))
    _raises(r"s_bin must have shape \[5\]", fc.fcat_spectral, torch.zeros((10, M)), sp, s_bin=torch.ones(4))
    _raises("must be on a GPU", fc.fcat_spectral, torch.zeros((10, M)), sp)
    _raises("one kernel per group of Y", fc.fcat_psf, torch.zeros((A, G + 1, NV, NU)), pb.psf)
    _raises(r"Y must have shape", fc.fcat_psf, torch.zeros((G, NV, NU)), pb.psf)
    _raises(r"out must have shape \[3\]\[4\]\[16\]", fc.fcat_pathlengths, pb, M, out=torch.zeros((A, NV, NU, M + 1)))
    _raises(r"scale must have shape \[2\]", fc.fcat_poisson, torch.zeros((A, G, NV * NU)), torch.ones(3), 1)
    _raises(r"flood must have shape \[4\]\[16\]", fc.fcat_log_projection, torch.ones((A, NV, NU)),
            torch.ones((NV, NU + 1)))
    _raises(r"energy must have shape \[5\]", fc.fcat_dose, pb, torch.ones(E - 1), torch.ones(E), 1.0)
    _raises(r"proj must have shape \[\*\]\[4\]\[16\]", fc.fcat_fdk_filter, pb.geometry, torch.ones((A, NU, NV)))
    import synth
    grid = synth.Grid(nx=8, ny=8, nz=2, dx=1.0, dy=1.0, dz=1.0)
    _raises(r"proj must have shape \[3\]\[4\]\[16\]", fc.fcat_fdk, pb.geometry, torch.ones((A - 1, NV, NU)), grid)
    _raises(r"volume must have shape \[2\]\[8\]\[8\]", fc.fcat_fdk, pb.geometry, torch.ones((A, NV, NU)), grid,
            volume=torch.zeros((2, 8, 9)))
    _raises("kernel must be square", fc.fcat_richardson_lucy, torch.ones((2, NV, NU)), torch.ones((5, 3)), 2)
    _raises("images must be torch.float32", fc.fcat_richardson_lucy, torch.ones((2, NV, NU), dtype=torch.float16),
            torch.ones((5, 5)), 2)


def test_surrogate_entry_points():
    pb = _problem()
    sp = pb.spectral
    P = 64 * M + 64 + 64 * 64 + 64 + G * 64 + G
    sur = fc.Surrogate(params=torch.zeros(P), in_scale=torch.ones(M), out_scale=torch.ones(G),
                       lin=torch.zeros((G, M)))
    _raises(r"Yprim must have shape \[2\]\[10\]", fc.fcat_mlp_gradients, sur, sp, torch.zeros((10, M)),
            torch.zeros((G, 11)))
    bad = fc.Surrogate(params=torch.zeros(P - 1), in_scale=torch.ones(M), out_scale=torch.ones(G),
                       lin=torch.zeros((G, M)))
    _raises(r"surrogate.params must have shape", fc.fcat_mlp_forward, bad, sp, torch.zeros((10, M)))
    _raises("must be on a GPU", fc.fcat_mlp_forward, sur, sp, torch.zeros((10, M)))
    tr = fc.MlpTrain(params=torch.zeros(P), adam_m=torch.zeros(P), adam_v=torch.zeros(P - 1))
    _raises("train.adam_v must have shape", fc.fcat_mlp_train_epoch, tr, sur, sp, torch.zeros((10, M)),
            torch.zeros((G, 10)), torch.zeros(10, dtype=torch.int32), 4)
    tr = fc.MlpTrain(params=torch.zeros(P), adam_m=torch.zeros(P), adam_v=torch.zeros(P))
    _raises("order must be torch.int32", fc.fcat_mlp_train_epoch, tr, sur, sp, torch.zeros((10, M)),
            torch.zeros((G, 10)), torch.zeros(10, dtype=torch.int64), 4)
