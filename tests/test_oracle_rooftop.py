"""The rooftop/pulse oracle (oracle/rooftop.py): its FFT product equals the
brute-force sums, its matrix is complex symmetric (reciprocity; a dropped
or mis-signed difference operator breaks it), its face contrast follows the
normal-flux continuity reading, and the discretisation converges to the Mie
series (Sec. III, Figs. 1-2)."""
import numpy as np
import pytest

import workloads as W
from oracle import operator as op, physics, rooftop as rt


def _padded_random(seed, shape, spacing):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    eps = np.ones(shape, complex)
    inner = (nz - 2, ny - 2, nx - 2)
    fill = rng.random(inner) < 0.8
    eps[1:-1, 1:-1, 1:-1] = np.where(fill, 1.5 + 3 * rng.random(inner) - 0.5j * rng.random(inner), 1.0)
    return op.Grid(nx, ny, nz, *spacing, 1.0, eps)


@pytest.mark.parametrize("shape,spacing", [((6, 7, 8), (0.05, 0.07, 0.06)), ((5, 5, 5), (0.04, 0.04, 0.04)),
                                           ((8, 4, 6), (0.08, 0.03, 0.05))])
def test_fft_product_equals_direct_sums(shape, spacing):
    g = _padded_random(sum(shape), shape, spacing)
    rng = np.random.default_rng(3)
    P = rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)
    fm = rt.face_mask(g)
    P = P * fm
    a = rt.RooftopFFT(g).scatter(P)
    b = rt.scatter_direct(g, P)
    assert np.abs((a - b)[fm]).max() <= 1e-12 * np.abs(b[fm]).max()
    c = rt.RooftopFFT(g, pad=3).scatter(P)   # any embedding length >= 2n
    assert np.abs((c - b)[fm]).max() <= 1e-12 * np.abs(b[fm]).max()


@pytest.mark.parametrize("shape,spacing", [((5, 6, 6), (0.05, 0.07, 0.06)), ((6, 5, 5), (0.04, 0.04, 0.04))])
def test_matrix_is_complex_symmetric(shape, spacing):
    """grad = -div^T makes the grad-div part symmetric; a sign or index
    mistake in either difference operator breaks the symmetry."""
    g = _padded_random(7 * sum(shape), shape, spacing)
    A, _ = rt.dense_matrix(g)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(A - A.conj().T).max() > 1e-6 * np.abs(A).max()   # not Hermitian


def test_face_contrast_reading():
    """Normal-flux continuity: a face between eps 1 and eps e has contrast
    (1 - m)/m, m = (1 + 1/e)/2; between two cells of eps e it is e - 1; a
    face of two vacuum cells has no unknown."""
    eps = np.ones((3, 3, 4), complex)
    eps[1, 1, 1] = eps[1, 1, 2] = 4.0
    g = op.Grid(4, 3, 3, 1.0, 1.0, 1.0, 1.0, eps)
    c = rt.face_chi(g)
    m = 0.5 * (1 + 0.25)
    assert c[0, 1, 1, 0] == pytest.approx((1 - m) / m)       # vacuum | 4
    assert c[0, 1, 1, 1] == pytest.approx(3.0)               # 4 | 4
    assert c[0, 1, 1, 2] == pytest.approx((1 - m) / m)       # 4 | vacuum
    assert c[1, 0, 0, 0] == 0 and not rt.face_mask(g)[2, 0, 0, 0]


def test_boundary_layers_must_be_vacuum():
    eps = np.ones((4, 4, 4), complex)
    eps[0, 1, 1] = 2.0
    with pytest.raises(ValueError):
        rt.RooftopFFT(op.Grid(4, 4, 4, 1.0, 1.0, 1.0, 1.0, eps))


def _rcs_error(r, eps):
    lam = r * 40 / 8          # k a = 2 pi / 5, as the collocated Mie tests
    g = op.Grid.from_case(W.sphere(r, lam, eps, pad=1))
    P, info = rt.solve(g, rt.plane_wave(g), 1e-9, 5000)
    assert info.status == "converged"
    th = np.radians(np.arange(0, 181))
    rv = rt.rcs_eplane(g, P, th)
    rm = physics.mie_rcs_eplane(eps, r, lam, th)
    return float(np.linalg.norm(rv - rm) / np.linalg.norm(rm))


def test_rooftop_sphere_matches_mie():
    """E-plane RCS of a voxelised dielectric sphere (eps 2.25, 8 cells per
    radius) within 3% of the Mie series, and of a lossy metal sphere
    (eps -1.05 - 5.62j) within 6% at 8 and 4% at 12 cells per radius."""
    assert _rcs_error(8, 2.25) <= 0.03
    e8, e12 = _rcs_error(8, -1.05 - 5.62j), _rcs_error(12, -1.05 - 5.62j)
    assert e8 <= 0.06 and e12 <= 0.04 and e12 < e8
