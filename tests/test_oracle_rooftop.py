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


def test_face_owner_reading():
    """A face belongs to the block of its lower cell when that cell is a
    scatterer cell, else to the block of its upper cell; faces between
    vacuum cells have no owner."""
    eps = np.ones((3, 3, 6), complex)
    eps[1, 1, 1:3] = 2.0
    eps[1, 1, 3] = 3.0
    bid = np.full(eps.shape, -1)
    bid[1, 1, 1:3] = 0
    bid[1, 1, 3] = 1
    g = op.Grid(6, 3, 3, 1.0, 1.0, 1.0, 1.0, eps)
    own = rt.face_owner(g, bid)
    assert list(own[0, 1, 1, :]) == [0, 0, 0, 1, -1, -1]
    assert own[2, 0, 1, 3] == 1 and own[2, 1, 1, 3] == 1     # below (vacuum) and above cell 3
    assert own[1, 0, 0, 2] == -1


def _blocked(seed, interior, n_blocks):
    return W.padded(W.random_tiny(seed, interior, fill=0.8, n_blocks=n_blocks))


def test_rooftop_block_preconditioner_is_the_dense_block_inverse():
    """K2 = blockdiag(R_k A R_k^T) from the dense matrix: block_matvec equals
    K2 x, and the preconditioner at a tight inner tolerance equals K2^{-1} w
    (a wrong owner or a leaked coupling between blocks fails both)."""
    case = _blocked(31, (3, 3, 4), 3)
    g = op.Grid.from_case(case)
    A, idx = rt.dense_matrix(g)
    owner = rt.face_owner(g, case.block_id)[idx]
    K2 = np.where(owner[:, None] == owner[None, :], A, 0.0)
    M = rt.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-14, 500)
    assert len(M.blocks) == case.n_blocks >= 2
    rng = np.random.default_rng(32)
    x = np.zeros((3,) + case.shape, complex)
    x[idx] = rng.standard_normal(len(idx[0])) + 1j * rng.standard_normal(len(idx[0]))
    assert np.abs(M.block_matvec(x)[idx] - K2 @ x[idx]).max() <= 1e-12 * np.abs(K2 @ x[idx]).max()
    want = np.linalg.solve(K2, x[idx])
    assert np.abs(M(x)[idx] - want).max() <= 1e-9 * np.abs(want).max()


def test_rooftop_preconditioned_solve():
    """The preconditioned solve reaches the unique solution of the plain one;
    with every face in one block and exact inner solves it takes one step."""
    case = _blocked(33, (4, 5, 4), 3)
    g = op.Grid.from_case(case)
    e = rt.plane_wave(g)
    P0, i0 = rt.solve(g, e, 1e-11, 2000)
    P1, i1, M = rt.solve_preconditioned(g, e, case.block_id, case.n_blocks, 1e-11, 500, 1e-4, 500)
    assert i0.status == i1.status == "converged" and i1.iterations < i0.iterations
    assert np.abs(P1 - P0).max() <= 1e-8 * np.abs(P0).max()
    one = np.where(g.mask, 0, -1)
    _, i2, _ = rt.solve_preconditioned(g, e, one, 1, 1e-8, 50, 1e-13, 500)
    assert i2.status == "converged" and i2.iterations == 1


def test_sparse_direct_evaluation_equals_the_fft_operator():
    """rooftop.apply_at (direct sums over a sparse P, any grid size) equals
    the FFT operator at sampled faces, sources and far faces alike."""
    c = W.padded(W.random_tiny(5, (5, 6, 7), fill=0.7))
    g = op.Grid.from_case(c)
    rng = np.random.default_rng(1)
    idx = np.argwhere(rt.face_mask(g))
    src = idx[rng.choice(len(idx), 25, replace=False)]
    vals = rng.standard_normal(25) + 1j * rng.standard_normal(25)
    P = np.zeros((3,) + c.shape, complex)
    P[tuple(src.T)] = vals
    full = rt.RooftopFFT(g)(P)
    dst = np.argwhere(np.ones((3,) + c.shape, bool))[rng.choice(3 * c.nvox, 60, replace=False)]
    dst = np.concatenate([dst, src[:5]])
    got = rt.apply_at(g, src, vals, dst)
    assert np.abs(got - full[tuple(dst.T)]).max() <= 1e-13 * np.abs(full).max()
