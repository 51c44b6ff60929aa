"""Fields from a solution on the GPU (vie_total_field_box, vie_far_field,
vie_rcs) against the oracle.

* Total field at every box voxel vs the oracle's E_inc + sum T P (FP64 to
  1e-12, mixed to 1e-5), through both the row and the fused-plane product
  paths.
* Far field vs the oracle's direct sum for random currents (FP64, 1e-11).
* The Mie comparison of Sec. III run on the GPU: a voxelised sphere of
  radius 8 voxels at lambda = 40 voxels solved by libvie, its E-plane RCS
  from vie_rcs: equal to the oracle's RCS of the same currents (1e-10) and
  within the oracle's own tolerance of the Mie series (5% dielectric, 10%
  metal).
"""
import numpy as np
import pytest

import workloads as W
from oracle import operator as op, physics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2501_13512_amd import vie as V  # noqa: E402


def _grid(case):
    return V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.wavelength)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 6, 6), (5, 8, 8)])
@pytest.mark.parametrize("prec,tol", [(V.VIE_FP64, 1e-12), (V.VIE_MIXED, 1e-5)])
def test_total_field_box_matches_oracle(vie_ctx, shape, prec, tol):
    case = W.random_tiny(80 + shape[0], shape, fill=0.7)
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(81)
    P = (rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)) * g.mask
    e = physics.plane_wave(g, (0.0, 0.6, 0.8), (1.0, 0.0, 0.0))
    want = physics.total_field_box(g, P, e)
    Pr = V.Problem(_grid(case), case.eps, None, 0, ctx=vie_ctx)
    try:
        pd, ed = torch.from_numpy(P).cuda(), torch.from_numpy(e).cuda()
        out = torch.empty_like(pd)
        V.vie_total_field_box(Pr.handle, prec, pd, ed, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        Pr.close()
    assert _rel(got, want) <= tol


@pytest.mark.parametrize("shape", [(4, 5, 6), (7, 3, 9)])
def test_far_field_matches_oracle(vie_ctx, shape):
    case = W.random_tiny(90 + shape[0], shape, fill=0.8, spacing=(0.04, 0.05, 0.03))
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(91)
    P = (rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)) * g.mask
    d = rng.standard_normal((37, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    want = physics.far_field_vector(g, P, d)
    Pr = V.Problem(_grid(case), case.eps, None, 0, ctx=vie_ctx)
    try:
        got = V.vie_far_field(Pr.handle, torch.from_numpy(P).cuda(), d)
    finally:
        Pr.close()
    assert _rel(got, want) <= 1e-11


def test_far_field_rejects_non_unit_direction(vie_ctx):
    case = W.random_tiny(95, (3, 3, 3))
    Pr = V.Problem(_grid(case), case.eps, None, 0, ctx=vie_ctx)
    try:
        P = torch.zeros(3 * 27, dtype=torch.complex128, device="cuda")
        with pytest.raises(V.VieError) as e:
            V.vie_far_field(Pr.handle, P, np.array([[1.0, 1.0, 0.0]]))
        assert e.value.code == V.VIE_EINVAL
    finally:
        Pr.close()


@pytest.mark.parametrize("eps,tol_rcs", [(2.25, 0.05), (-1.05 - 5.62j, 0.10)])
def test_mie_comparison_on_gpu(vie_ctx, eps, tol_rcs):
    r, lam = 8, 40.0
    case = W.sphere(r, lam, eps)
    g = op.Grid.from_case(case)
    Pr = V.Problem(_grid(case), case.eps, None, 0, ctx=vie_ctx)
    try:
        e = torch.from_numpy(V.vie_plane_wave(Pr.grid, case.kdir, case.pol)).cuda()
        out = torch.empty_like(e)
        pol = torch.empty_like(e)
        st = V.vie_stats()
        o = V.make_opts(tol_outer=1e-10, maxit_outer=3000, precondition=False, precision=V.VIE_FP64)
        assert V.vie_solve_device(Pr.handle, e, o, out, pol, st) == V.VIE_OK
        th = np.radians(np.arange(0, 181))
        rh = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=-1)
        sigma = V.vie_rcs(Pr.handle, pol, rh)
        Pn = pol.cpu().numpy()
    finally:
        Pr.close()
    assert _rel(sigma, physics.rcs_eplane(g, Pn, th)) <= 1e-10
    mie = physics.mie_rcs_eplane(eps, r, lam, th)
    assert _rel(sigma, mie) <= tol_rcs
