"""Pins of the oracle's solver (Sec. II-B, eqs. (10)-(11)).

* BiCGSTAB iterates equal those of an independent library implementation of
  the same van der Vorst recurrence (scipy), with and without a right
  preconditioner, iteration by iteration.
* Converged solutions equal the dense LU solution.
* Special cases of the block preconditioner: one block solved exactly gives
  convergence in one outer step; single-voxel blocks reduce to the explicit
  3x3 block-Jacobi inverse; every partition reaches the same solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import green, krylov, operator as op, physics


def _problem(seed, shape, fill=0.8, n_blocks=2):
    case = W.random_tiny(seed, shape, fill=fill, n_blocks=n_blocks)
    g = op.Grid.from_case(case)
    return case, g, physics.plane_wave(g)


@pytest.mark.parametrize("precondition", [False, True])
def test_iterates_match_scipy_bicgstab(precondition):
    n4 = 4
    kk, jj, ii = np.meshgrid(*[np.arange(n4)] * 3, indexing="ij")
    g = op.Grid(n4, n4, n4, 0.06, 0.06, 0.06, 1.0, np.full((n4,) * 3, 4.0 + 0j))
    block_id = (ii >= 2).astype(np.int32)
    e = physics.plane_wave(g)
    Z, idx = op.dense_matrix(g)
    A = lambda x: op.from_support(g, Z @ op.to_support(g, x, idx), idx)
    b = op.to_support(g, e * g.mask, idx)
    n = b.size
    if precondition:
        # fixed linear preconditioner: dense inverse of the block-diagonal
        # part of A (eq. (10)), the limit of the inner solves at zero tolerance
        i, j, k = idx
        blk = np.tile(block_id[k, j, i], 3)
        Minv = np.linalg.inv(np.where(blk[:, None] == blk[None, :], Z, 0))
        M_grid = lambda w: op.from_support(g, Minv @ op.to_support(g, w, idx), idx)
        M_s = spla.LinearOperator((n, n), matvec=lambda v: Minv @ v, dtype=complex)
    else:
        M_grid = None
        M_s = None
    A_s = spla.LinearOperator((n, n), matvec=lambda v: Z @ v, dtype=complex)
    hist = []
    spla.bicgstab(A_s, b, rtol=1e-30, atol=0.0, maxiter=8, M=M_s, callback=lambda xk: hist.append(xk.copy()))
    for k in range(1, 9):
        x, info = krylov.bicgstab(A, e * g.mask, 0.0, k, M_grid)
        assert info.iterations == k
        xs = op.to_support(g, x, idx)
        # identical arithmetic up to rounding order (a wrong step differs at
        # the 1e-2 level)
        tol = 1e-13
        assert np.linalg.norm(xs - hist[k - 1]) <= tol * np.linalg.norm(hist[k - 1])


@pytest.mark.parametrize("seed,shape", [(41, (3, 4, 5)), (42, (5, 5, 5)), (43, (2, 6, 3))])
def test_converged_bicgstab_matches_dense_lu(seed, shape):
    case, g, e = _problem(seed, shape)
    Pd = krylov.solve_dense(g, e)
    s = krylov.solve(g, e, 1e-13, 2000)
    assert s.info.status == "converged"
    assert np.linalg.norm(s.P - Pd) <= 1e-10 * np.linalg.norm(Pd)
    sp = krylov.solve(g, e, 1e-13, 2000, case.block_id, case.n_blocks, 1e-6, 500)
    assert sp.info.status == "converged"
    assert np.linalg.norm(sp.P - Pd) <= 1e-10 * np.linalg.norm(Pd)


def test_single_exact_block_converges_in_one_step():
    case, g, e = _problem(51, (4, 3, 4))
    bid = np.where(g.mask, 0, -1).astype(np.int32)
    s = krylov.solve(g, e, 1e-8, 50, bid, 1, 1e-14, 2000)
    assert s.info.status == "converged"
    assert s.info.iterations == 1 and s.info.half_step


def test_single_voxel_blocks_are_block_jacobi():
    case, g, e = _problem(52, (3, 3, 4))
    bid = np.full(case.shape, -1, np.int32)
    ids = np.arange(int(g.mask.sum()), dtype=np.int32)
    bid[g.mask] = ids
    pre = krylov.BlockPreconditioner(g, bid, ids.size, 1e-15, 100)
    rng = np.random.default_rng(0)
    w = (rng.standard_normal((3,) + case.shape) + 1j * rng.standard_normal((3,) + case.shape)) * g.mask
    y = pre(w)
    t0 = green.self_term(g.dx, g.dy, g.dz, g.k0)
    want = w / (g.chi_inv - t0) * g.mask
    want[:, ~g.mask] = 0
    assert np.linalg.norm(y - want) <= 1e-13 * np.linalg.norm(want)


def test_zero_rhs_block_returns_zero():
    case, g, e = _problem(53, (3, 3, 3), n_blocks=3)
    pre = krylov.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-6, 100)
    w = np.zeros((3,) + case.shape, complex)
    assert np.all(pre(w) == 0)
    assert pre.inner_counts[-1] == [0] * len(pre.blocks)


def test_zero_rhs_outer_is_zero_iterations():
    case, g, e = _problem(54, (2, 2, 2))
    s = krylov.solve(g, np.zeros_like(e), 1e-6, 10)
    assert s.info.iterations == 0 and np.all(s.P == 0)


def test_iteration_cap_keeps_last_iterate():
    case, g, e = _problem(55, (4, 4, 4))
    s = krylov.solve(g, e, 1e-14, 3)
    assert s.info.status == "not_converged" and s.info.iterations == 3
    x3, _ = krylov.bicgstab(op.FFTOperator(g), e * g.mask, 0.0, 3)
    assert np.array_equal(s.P, x3)


def test_block_preconditioner_reduces_outer_steps_cube16():
    """Table II / Sec. III-A: the block preconditioner cuts outer steps."""
    case = W.cube16()
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g)
    plain = krylov.solve(g, e, case.tol_outer, case.maxit_outer)
    pre = krylov.solve(g, e, case.tol_outer, case.maxit_outer, case.block_id, case.n_blocks,
                       case.tol_inner, case.maxit_inner)
    assert plain.info.status == pre.info.status == "converged"
    assert pre.info.iterations < plain.info.iterations
    diff = np.linalg.norm(plain.E_tot - pre.E_tot) / np.linalg.norm(plain.E_tot)
    assert diff <= 50 * case.tol_outer
