"""The configuration files: one JSON per configuration (geometry, grid,
seed, materials, energy bins, groups, optical-spread size, projector form),
each loading into the arrays it describes."""
import glob
import json
import os

import numpy as np
import pytest

import synth

FILES = sorted(glob.glob(os.path.join(synth.CONFIG_DIR, "*.json")))


def test_every_configuration_has_a_file():
    names = {os.path.basename(f) for f in FILES}
    assert set(synth.CONFIG_FILES.values()) <= names
    modes = {json.load(open(f))["mode"] for f in FILES}
    assert modes == {"plain", "split_bf16", "surrogate"}


@pytest.mark.parametrize("path", [f for f in FILES if "head" not in f], ids=os.path.basename)
def test_file_describes_the_loaded_arrays(path):
    p = json.load(open(path))
    cfg = synth.load_config(path)
    g, ph, s = cfg.geometry, cfg.phantom, cfg.spectral
    assert (g.sid, g.sdd, g.nu, g.nv, g.du, g.dv, g.n_angles) == tuple(
        p["geometry"][k] for k in ("sid_mm", "sdd_mm", "nu", "nv", "du_mm", "dv_mm", "n_angles"))
    assert ph.labels.shape == (p["grid"]["nz"], p["grid"]["ny"], p["grid"]["nx"])
    assert (ph.dx, ph.dy, ph.dz) == (p["grid"]["dx_mm"], p["grid"]["dy_mm"], p["grid"]["dz_mm"])
    assert s.mu.shape == (len(p["materials"]), p["energy"]["bins"]) and s.n_groups == p["groups"]
    assert list(s.material_names) == p["materials"] and cfg.mode == p["mode"]
    e = p["energy"]
    np.testing.assert_allclose(s.energies[[0, -1]], [e["first"], e["first"] + e["span"]], rtol=1e-12)
    assert set(np.unique(ph.labels)) <= set(range(len(p["materials"])))
    assert (cfg.psf is None) == (p["psf_k"] == 0) and (cfg.scatter is None) == (not p["scatter"])
    if cfg.psf is not None:
        assert cfg.psf.kernels.shape == (p["groups"], p["psf_k"], p["psf_k"])
    if cfg.scatter is not None:
        assert cfg.scatter.maps([0]).shape == (1, g.nv, g.nu)


def test_an_edited_file_gives_a_smaller_workload():
    p = json.load(open(os.path.join(synth.CONFIG_DIR, "tiny.json")))
    p["geometry"].update(n_angles=12, nu=40)
    p["energy"].update(bins=9)
    cfg = synth.load_config(p)
    assert cfg.geometry.n_angles == 12 and cfg.geometry.nu == 40 and cfg.spectral.n_energy == 9
    # the seed fixes the phantom: the grid is unchanged, so are the labels
    np.testing.assert_array_equal(cfg.phantom.labels, synth.make_config(1).phantom.labels)
    with pytest.raises(ValueError, match="unknown recipe"):
        synth.load_config(dict(p, recipe="knee"))
