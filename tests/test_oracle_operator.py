"""Pins of the oracle's VIE operator (eqs. (2)-(4), (6)).

* The FFT product equals the brute-force O(N^2) sum on every tiny grid
  shape (this is what the Toeplitz + FFT statement of Sec. I promises).
* The assembled matrix is complex symmetric (reciprocity).
* One voxel reduces to the textbook Clausius-Mossotti polarisability in
  the quasi-static limit.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import green, operator as op


def _rand_vec(rng, shape):
    return rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)


SHAPES = sorted(set(itertools.product((1, 2, 3, 5, 6), repeat=3)))[::3] + [(6, 6, 6), (1, 1, 1), (1, 6, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fft_matches_direct(shape):
    seed = 100 + shape[0] * 36 + shape[1] * 6 + shape[2]
    case = W.random_tiny(seed, shape, fill=0.75)
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(seed)
    x = _rand_vec(rng, case.shape) * g.mask
    a = op.matvec_direct(g, x)
    b = op.matvec_fft(g, x)
    scale = max(np.linalg.norm(a), 1e-300)
    assert np.linalg.norm(a - b) <= 1e-13 * scale


def test_fft_matches_direct_noncubic_spacing_and_long_axis():
    case = W.random_tiny(7, (2, 3, 9), fill=0.9, spacing=(0.02, 0.05, 0.11), wavelength=0.8)
    g = op.Grid.from_case(case)
    x = _rand_vec(np.random.default_rng(3), case.shape) * g.mask
    a = op.matvec_direct(g, x)
    b = op.matvec_fft(g, x)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_dense_matrix_matches_direct():
    case = W.random_tiny(11, (3, 4, 4), fill=0.6)
    g = op.Grid.from_case(case)
    Z, idx = op.dense_matrix(g)
    x = _rand_vec(np.random.default_rng(1), case.shape) * g.mask
    want = op.matvec_direct(g, x)
    got = op.from_support(g, Z @ op.to_support(g, x, idx), idx)
    assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want)


def test_complex_symmetry_reciprocity():
    case = W.random_tiny(12, (4, 3, 5), fill=0.8)
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(5)
    u = _rand_vec(rng, case.shape) * g.mask
    v = _rand_vec(rng, case.shape) * g.mask
    Au = op.matvec_fft(g, u)
    Av = op.matvec_fft(g, v)
    lhs = np.sum(u * Av)
    rhs = np.sum(v * Au)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_vacuum_voxels_are_masked():
    case = W.random_tiny(13, (3, 3, 3), fill=0.5)
    g = op.Grid.from_case(case)
    x = _rand_vec(np.random.default_rng(2), case.shape)     # NOT masked on input
    y = op.matvec_fft(g, x)
    assert np.all(y[:, ~g.mask] == 0)
    assert np.allclose(y, op.matvec_fft(g, x * g.mask), rtol=0, atol=0)


@pytest.mark.parametrize("chi", [3.0, 1.25, -2.05 - 5.62j])
def test_single_voxel_clausius_mossotti(chi):
    """P = E_inc / (1/chi - T(0)) -> 3 chi / (chi + 3) E_inc as k0 d -> 0."""
    eps = np.full((1, 1, 1), 1.0 + chi, dtype=complex)
    for d in [1e-2, 1e-3]:
        g = op.Grid(1, 1, 1, d, d, d, 1.0, eps)
        e = np.zeros((3, 1, 1, 1), complex)
        e[0] = 1.0
        Z, idx = op.dense_matrix(g)
        P = np.linalg.solve(Z, op.to_support(g, e, idx))[0]
        cm = 3 * chi / (chi + 3)
        x = g.k0 * (3 * d ** 3 / (4 * np.pi)) ** (1 / 3)
        assert abs(P - cm) <= 2 * abs(cm) * abs(cm) * x * x + 1e-14


def test_embedding_length_does_not_change_product():
    """Any circulant length >= 2n - 1 gives the same convolution."""
    case = W.random_tiny(21, (5, 4, 3), fill=0.8)
    g = op.Grid.from_case(case)
    x = _rand_vec(np.random.default_rng(9), case.shape) * g.mask
    ref = op.FFTOperator(g).convolve(x)
    import scipy.fft
    for L in [(5, 7, 9), (8, 12, 16), (6, 9, 10)]:
        kern = green.embedded_kernel(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.k0, L)
        S = scipy.fft.fftn(kern, axes=(1, 2, 3))
        xp = np.zeros((3, L[2], L[1], L[0]), complex)
        xp[:, :g.nz, :g.ny, :g.nx] = x
        X = scipy.fft.fftn(xp, axes=(1, 2, 3))
        Y = np.zeros_like(X)
        for c, (a, b) in enumerate(green.COMPONENTS):
            Y[a] += S[c] * X[b]
            if a != b:
                Y[b] += S[c] * X[a]
        y = scipy.fft.ifftn(Y, axes=(1, 2, 3))[:, :g.nz, :g.ny, :g.nx]
        assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)


def test_c64_product_mode_is_single_precision_of_the_same_operator():
    """The complex64 product differs from FP64 by single-precision rounding
    only (relative ~1e-7), and keeps the FP64 local term exactly."""
    case = W.random_tiny(61, (9, 8, 7), fill=0.8)
    g = op.Grid.from_case(case)
    x = _rand_vec(np.random.default_rng(6), case.shape) * g.mask
    a = op.FFTOperator(g)(x)
    b = op.FFTOperator(g, product="c64")(x)
    err = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-9 < err < 1e-5
    local = x * g.chi_inv
    ca = op.FFTOperator(g).convolve(x)
    cb = op.FFTOperator(g, product="c64").convolve(x)
    assert np.linalg.norm((local - cb) * g.mask - b) <= 1e-15 * np.linalg.norm(b)
    assert np.linalg.norm(ca - cb) / np.linalg.norm(ca) < 1e-5


def test_sparse_direct_evaluation_equals_the_direct_product():
    """operator.apply_at (direct sums over a sparse x, any grid size) equals
    the all-pairs direct product at sampled voxels, sources included."""
    import workloads as W
    c = W.random_tiny(6, (5, 6, 7), fill=0.7)
    g = op.Grid.from_case(c)
    rng = np.random.default_rng(2)
    vox = np.argwhere(np.ones(c.shape, bool))
    src = vox[rng.choice(len(vox), 30, replace=False)]
    xs = rng.standard_normal((30, 3)) + 1j * rng.standard_normal((30, 3))
    x = np.zeros((3,) + c.shape, complex)
    for k in range(3):
        x[k][tuple(src.T)] = xs[:, k]
    full = op.matvec_direct(g, x)
    dst = np.concatenate([vox[rng.choice(len(vox), 50, replace=False)], src[:5]])
    got = op.apply_at(g, src, xs, dst)
    want = np.stack([full[k][tuple(dst.T)] for k in range(3)], axis=1)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(full).max()
