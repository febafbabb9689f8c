"""Input problems noted by fcat_project while it runs, reported by
fcat_project_status (labels outside 0..n_mat-1 of Sec. II.C, non-finite
tables), without a host synchronisation inside the projector call.

Documented outputs: a voxel with an out-of-range label adds no path length
to any material, which is the projection of the same phantom with that
voxel given an extra material of zero attenuation (the oracle computes
that one); a NaN in mu reaches the rays that cross the material and no
others.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import rel_err

pytestmark = pytest.mark.gpu

LABEL_RANGE, NONFINITE = 3, 4


def _status(fc, ws):
    try:
        fc.fcat_project_status(ws)
    except fc.FcatError as e:
        return e.status
    return 0


def _ws(fc, pb, mode="plain"):
    return torch.empty(fc.fcat_project_workspace_bytes(pb, mode), dtype=torch.uint8, device="cuda")


def test_out_of_range_labels_are_reported_and_add_no_length(fc):
    cfg = synth.make_config(1)
    M = cfg.spectral.n_mat
    lab = cfg.phantom.labels.copy()
    lab[4:12, 28:36, 28:36] = M           # one past the last material, inside the water cylinder
    lab[0:3, 10:14, 40:44] = -3           # negative, in air at the edge
    cfg.phantom.labels = lab
    pb = fc.upload(cfg)
    ws = _ws(fc, pb)
    out = fc.fcat_project(pb, workspace=ws).cpu().numpy()     # returns OK: nothing is known yet
    assert _status(fc, ws) == LABEL_RANGE
    # reference: the bad voxels as an extra material with mu = 0
    ref_cfg = copy.deepcopy(cfg)
    ref_cfg.phantom.labels = np.where((lab < 0) | (lab >= M), M, lab).astype(np.int8)
    ref_cfg.spectral.mu = np.concatenate([cfg.spectral.mu, np.zeros((1, cfg.spectral.n_energy))]).astype(
        cfg.spectral.mu.dtype)
    angles = [0, 11, 22, 33]
    ref = oracle.project(ref_cfg, angles)
    err = rel_err(out[angles], ref)
    print(f"bad labels: max rel err vs zero-attenuation reading {err.max():.3e}")
    assert err.max() <= 1e-5
    # the flags are cleared by the next call on the same workspace
    pb_ok = fc.upload(synth.make_config(1))
    fc.fcat_project(pb_ok, workspace=ws)
    assert _status(fc, ws) == 0


@pytest.mark.parametrize("mode", ["plain", "split_bf16"])
def test_nan_mu_is_reported_and_propagates(fc, mode):
    cfg = synth.make_config(1)
    pb = fc.upload(cfg)
    ws = _ws(fc, pb, mode)
    clean = fc.fcat_project(pb, mode=mode, workspace=ws).cpu().numpy()
    assert _status(fc, ws) == 0 and np.isfinite(clean).all()
    m_bad = 2                                   # a cylindrical insert
    pb.spectral.mu[m_bad, 5] = float("nan")
    out = fc.fcat_project(pb, mode=mode, workspace=ws).cpu().numpy()
    assert _status(fc, ws) == NONFINITE
    # the contraction multiplies the NaN by every hit ray's path length in
    # that material, zero or not: the hit rays' outputs are NaN
    L = fc.fcat_pathlengths(pb, cfg.spectral.n_mat).cpu().numpy()
    hit = L.sum(-1) > 0
    assert np.isnan(out[hit]).all()


def test_nan_scatter_flood_and_psf_are_reported(fc):
    rng = np.random.default_rng(3)
    cfg = synth.make_config(1)
    g = cfg.geometry
    cfg.scatter = synth.scatter_blobs(rng, g.n_angles, g.nu, g.nv, (30, 60), (4, 8))
    cfg.psf = synth.Psf(synth.gaussian_psfs(rng, 1, 15))
    pb = fc.upload(cfg)
    ws = _ws(fc, pb)
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == 0
    pb.scatter.maps[7, 3, 5] = float("inf")
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == NONFINITE
    pb.scatter.maps[7, 3, 5] = 0.0
    pb.spectral.flood = torch.ones((g.nv, g.nu), dtype=torch.float32, device="cuda")
    pb.spectral.flood[2, 2] = float("nan")
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == NONFINITE
    pb.spectral.flood = None
    pb.psf.kernels[0, 7, 7] = float("nan")
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == NONFINITE
    pb.psf.kernels[0, 7, 7] = 0.1
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == 0


def test_label_range_is_reported_first_and_project_check_raises(fc):
    cfg = synth.make_config(1)
    lab = cfg.phantom.labels.copy()
    lab[8, 32, 32] = 100
    cfg.phantom.labels = lab
    pb = fc.upload(cfg)
    pb.spectral.phi[0] = float("nan")
    ws = _ws(fc, pb)
    fc.fcat_project(pb, workspace=ws)
    assert _status(fc, ws) == LABEL_RANGE
    with pytest.raises(fc.FcatError) as e:
        fc.project(pb.geometry, pb.phantom, pb.spectral.mu, pb.spectral.phi, pb.spectral.eta)
    assert e.value.status == LABEL_RANGE
