"""GPU parity of the image projector A and its transpose A^T with the oracle.

Tolerances from the FP32 arithmetic: each plane crossing is a distance t
rounded once in FP32, so a segment's length is off by at most about two ulps
of the largest distance on the ray, 2^-22 t_end; the image projector sums
f_k l_k, whose error is then at most (number of segments) 2^-22 t_end
max|f| (compensated sum), and the back-projection's voxel values are off by
the same per-segment amount times y.  With the test grids' rays (at most
about 100 segments, t_end below 100 mm) that is below 2e-4 of the largest
projection for an image of random values, and far below it for a smooth
image, where errors of neighbouring segments cancel.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _setup(nx=40, ny=36, nz=20, A=12):
    geo = synth.Geometry(sid=300.0, sdd=450.0, nu=96, nv=40, du=0.9, dv=0.9, n_angles=A, off_u=0.37, off_v=-0.21)
    grid = synth.Grid(nx=nx, ny=ny, nz=nz, dx=1.0, dy=1.1, dz=0.9, cx=0.3, cy=-0.2, cz=0.1)
    return geo, grid


def _smooth(grid, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    f = np.zeros((grid.nz, grid.ny, grid.nx))
    for _ in range(5):
        c = rng.uniform([0, 0, 0], [grid.nz, grid.ny, grid.nx])
        s = rng.uniform(3, 9)
        f += rng.uniform(0.2, 1.0) * np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2) / (2 * s * s))
    return f.astype(np.float32)


def _dev(fc, a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _pb(fc, geo):
    return fc.Geometry(geo.sid, geo.sdd, geo.nu, geo.nv, geo.du, geo.dv, geo.n_angles, geo.off_u, geo.off_v)


@pytest.mark.parametrize("kind", ["smooth", "random"])
def test_image_projection_matches_oracle(fc, kind):
    geo, grid = _setup()
    f = _smooth(grid, 1) if kind == "smooth" else \
        np.random.default_rng(2).uniform(0, 2, size=(grid.nz, grid.ny, grid.nx)).astype(np.float32)
    got = fc.fcat_image_project(_pb(fc, geo), grid, _dev(fc, f)).cpu().numpy()
    ref = oracle.forward_image(geo, grid, f, range(geo.n_angles))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"A f ({kind}): max |err| / max |ref| = {err:.2e}")
    assert err <= (1e-5 if kind == "smooth" else 2e-4)
    # an angle sub-range gives the same rows
    part = fc.fcat_image_project(_pb(fc, geo), grid, _dev(fc, f), 5, 9).cpu().numpy()
    np.testing.assert_array_equal(part, got[5:9])


def test_image_backprojection_matches_oracle_and_accumulates(fc):
    geo, grid = _setup()
    rng = np.random.default_rng(3)
    y = (1.0 + 0.5 * np.sin(np.linspace(0, 3, geo.nu))[None, None, :]
         * rng.uniform(0.5, 1.0, size=(geo.n_angles, geo.nv, 1))).astype(np.float32)
    got = fc.fcat_image_backproject(_pb(fc, geo), grid, _dev(fc, y)).cpu().numpy()
    ref = oracle.backproject_image(geo, grid, y, range(geo.n_angles))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"A^T y: max |err| / max |ref| = {err:.2e}")
    assert err <= 1e-4
    # two angle halves accumulated give the whole
    img = fc.fcat_image_backproject(_pb(fc, geo), grid, _dev(fc, y[:5]), 0)
    img = fc.fcat_image_backproject(_pb(fc, geo), grid, _dev(fc, y[5:]), 5, image=img, accumulate=True)
    np.testing.assert_allclose(img.cpu().numpy(), got, rtol=1e-5, atol=1e-6 * np.abs(got).max())


def test_adjoint_identity_on_the_gpu(fc):
    geo, grid = _setup(nx=48, ny=44, nz=24, A=16)
    rng = np.random.default_rng(4)
    f = rng.normal(size=(grid.nz, grid.ny, grid.nx)).astype(np.float32)
    y = rng.normal(size=(geo.n_angles, geo.nv, geo.nu)).astype(np.float32)
    Af = fc.fcat_image_project(_pb(fc, geo), grid, _dev(fc, f)).cpu().numpy().astype(np.float64)
    ATy = fc.fcat_image_backproject(_pb(fc, geo), grid, _dev(fc, y)).cpu().numpy().astype(np.float64)
    lhs, rhs = float((Af * y).sum()), float((f * ATy).sum())
    scale = float(np.abs(Af * y).sum())
    print(f"<Af, y> {lhs:.6e}, <f, A^T y> {rhs:.6e}, difference / sum |terms| {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_iterative_reconstruction_converges(fc):
    """SIRT (x <- x + C A^T (R (p - A x)), R = 1 / A 1, C = 1 / A^T 1) from
    projections of a voxelised water cylinder with a denser insert: the
    residual falls at every iteration and the image approaches the truth."""
    import torch
    geo = synth.Geometry(sid=200.0, sdd=300.0, nu=96, nv=12, du=1.0, dv=1.0, n_angles=60)
    grid = synth.Grid(nx=48, ny=48, nz=6, dx=1.0, dy=1.0, dz=1.0)
    z, y, x = np.meshgrid(np.arange(6), np.arange(48) - 23.5, np.arange(48) - 23.5, indexing="ij")
    truth = np.where(x * x + y * y < 20.0 ** 2, 0.02, 0.0) + np.where((x - 6) ** 2 + y * y < 5.0 ** 2, 0.03, 0.0)
    pg = _pb(fc, geo)
    p = fc.fcat_image_project(pg, grid, _dev(fc, truth))
    ones_img = torch.ones((6, 48, 48), device="cuda")
    R = 1.0 / torch.clamp(fc.fcat_image_project(pg, grid, ones_img), min=1e-6)
    C = 1.0 / torch.clamp(fc.fcat_image_backproject(pg, grid, torch.ones_like(p)), min=1e-6)
    xk = torch.zeros_like(ones_img)
    res = []
    for _ in range(40):
        r = p - fc.fcat_image_project(pg, grid, xk)
        res.append(float(r.norm()))
        xk = xk + C * fc.fcat_image_backproject(pg, grid, (R * r).contiguous())
    assert all(b < a for a, b in zip(res, res[1:]))
    t = torch.as_tensor(truth, dtype=torch.float32, device="cuda")
    err = float((xk - t)[:, 8:40, 8:40].abs().mean() / t[:, 8:40, 8:40].abs().mean())
    print(f"SIRT: residual {res[0]:.3e} -> {res[-1]:.3e}; mean relative image error {err:.3f}")
    assert res[-1] < 0.05 * res[0] and err < 0.1
