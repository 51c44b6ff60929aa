"""Pins of the oracle's solver (Sec. II-B, eqs. (10)-(11)).

* BiCGSTAB iterates equal those of an independent library implementation of
  the same van der Vorst recurrence (scipy), with and without a right
  preconditioner, iteration by iteration.
* CGS iterates equal scipy's (same recurrence, residual recomputed as
  b - A x), with and without a right preconditioner.
* Converged solutions (BiCGSTAB, CGS) equal the dense LU solution.
* Special cases of the block preconditioner: one block solved exactly gives
  convergence in one outer step; single-voxel blocks reduce to the explicit
  3x3 block-Jacobi inverse; every partition reaches the same solution.
* Mixed precision with refinement: complex64 products alone stall at the
  single-precision level of the true residual; the FP64 residual and the
  corrections carry the iterate to the dense LU solution at the requested
  tolerance; the reported true residual is that of the dense matrix; no
  correction means the plain complex64 run.
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


@pytest.mark.parametrize("seed,shape,precondition", [(41, (3, 4, 5), True), (44, (5, 4, 6), False),
                                                     (45, (4, 4, 4), True)])
def test_mixed_refinement_reaches_dense_lu(seed, shape, precondition):
    """The complex64 main loop ends (converged on its recursive residual, or
    at its cap: inexact complex64 inner solves vary from step to step) with a
    true (FP64) residual at the single-precision level (> 1e-8 here); with
    refinement the true residual meets 1e-11 and the iterate is the dense LU
    solution to 1e-9.  Refining with the complex64 product instead of the
    FP64 one could not get below the single-precision level, and a
    correction of the wrong sign would diverge."""
    case, g, e = _problem(seed, shape)
    Pd = krylov.solve_dense(g, e)
    blocks = (case.block_id, case.n_blocks) if precondition else (None, 0)
    # inner solves tight: with inexact ones (1e-2, 1e-3) BiCGSTAB stalls on
    # these random partitions in FP64 as well (the preconditioner varies)
    s = krylov.solve_mixed(g, e, 1e-11, 400, blocks[0], blocks[1], 1e-6, 500, max_refine=3)
    assert s.info.status in ("converged", "not_converged")
    assert s.true_history[0] > 1e-8
    assert 1 <= s.refine_steps <= 3 and s.relres_true <= 1e-11
    assert np.linalg.norm(s.P - Pd) <= 1e-9 * np.linalg.norm(Pd)
    # the reported true residual is that of the assembled matrix
    Z, idx = op.dense_matrix(g)
    b = op.to_support(g, e * g.mask, idx)
    dense = np.linalg.norm(b - Z @ op.to_support(g, s.P, idx)) / np.linalg.norm(b)
    assert abs(dense - s.relres_true) <= 1e-3 * s.relres_true + 1e-15
    # every correction at least halves the true residual (its tolerance is
    # min(0.5, tol / relres), plus single-precision product error)
    for a, b_ in zip(s.true_history, s.true_history[1:]):
        assert b_ <= 0.6 * a


def test_mixed_without_refinement_is_the_complex64_loop():
    case, g, e = _problem(46, (4, 3, 5))
    s = krylov.solve_mixed(g, e, 1e-9, 300, case.block_id, case.n_blocks, 1e-3, 200, max_refine=0)
    p = krylov.solve(g, e, 1e-9, 300, case.block_id, case.n_blocks, 1e-3, 200, product="c64")
    assert s.refine_steps == 0 and s.info.iterations == p.info.iterations
    assert np.array_equal(s.P, p.P)
    assert s.inner_counts == p.inner_counts


def test_mixed_refinement_stops_at_tolerance_and_cap():
    """No correction when the main loop's true residual already meets the
    tolerance; at most max_refine corrections otherwise."""
    case, g, e = _problem(47, (4, 4, 3))
    loose = krylov.solve_mixed(g, e, 1e-4, 500, max_refine=3)
    assert loose.refine_steps == 0 and loose.true_history[0] <= 1e-4
    capped = krylov.solve_mixed(g, e, 1e-15, 500, max_refine=1)
    assert capped.refine_steps == 1 and len(capped.true_history) == 2


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


# ------------------------------------------------------------------ FGMRES
def _dense_problem(seed, n=24):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def _min_residuals(Aop, b, kmax):
    """min over x in K_j(Aop, b) of ||b - Aop x|| / ||b||, j = 1..kmax, by
    least squares on an orthonormal basis of the explicit Krylov space."""
    out = []
    K = [b / np.linalg.norm(b)]
    for j in range(1, kmax + 1):
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        AQ = Aop @ Q
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        out.append(np.linalg.norm(b - AQ @ y) / np.linalg.norm(b))
        K.append(Aop @ K[-1])
        K[-1] = K[-1] / np.linalg.norm(K[-1])
    return np.array(out)


def test_fgmres_residuals_are_the_krylov_minimum():
    """Without restart and with K = I each step's residual is the minimum over
    the Krylov space (the defining property of GMRES)."""
    A, b = _dense_problem(1)
    x, info = krylov.fgmres(lambda v: A @ v, b, 1e-14, 8, restart=50)
    want = _min_residuals(A, b, 8)
    assert np.allclose(info.history, want, rtol=1e-8, atol=1e-14)


def test_fgmres_fixed_preconditioner_is_right_preconditioned_gmres():
    """A fixed linear M: the residuals are the Krylov minima of A M."""
    A, b = _dense_problem(2)
    rng = np.random.default_rng(3)
    Mm = np.diag(1.0 / np.diag(A)) + 0.05 * rng.standard_normal(A.shape)
    x, info = krylov.fgmres(lambda v: A @ v, b, 1e-14, 7, restart=50, precond=lambda w: Mm @ w)
    assert np.allclose(info.history, _min_residuals(A @ Mm, b, 7), rtol=1e-8, atol=1e-14)


def test_fgmres_exact_preconditioner_one_step():
    A, b = _dense_problem(4)
    Ainv = np.linalg.inv(A)
    x, info = krylov.fgmres(lambda v: A @ v, b, 1e-12, 10, precond=lambda w: Ainv @ w)
    assert info.iterations == 1 and info.status == "converged"
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_fgmres_restarted_and_flexible_converges_to_dense_solution():
    """Restart every 10 steps and a preconditioner that changes at every
    call (point Jacobi of the local term and the identity, alternately):
    still the dense solution, and the final residual is the tolerance."""
    case = W.random_tiny(31, (3, 4, 4), fill=0.8)
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g)
    A = op.FFTOperator(g)
    b = krylov.masked_rhs(g, e)
    t0 = green.self_term(g.dx, g.dy, g.dz, g.k0)
    jac = np.where(g.mask, 1.0 / (g.chi_inv - t0 + (~g.mask)), 0.0)
    calls = [0]

    def M(w):
        calls[0] += 1
        return w * (jac if calls[0] % 2 else 1.0)

    x, info = krylov.fgmres(A, b, 1e-12, 3000, restart=10, precond=M)
    assert info.status == "converged"
    ref = krylov.solve_dense(g, e)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    true = np.linalg.norm(b - A(x)) / np.linalg.norm(b)
    assert true <= 1e-11
    assert np.all(np.diff(info.history[:10]) <= 1e-15)   # monotone inside a cycle


def test_fgmres_zero_rhs():
    x, info = krylov.fgmres(lambda v: v, np.zeros(4, complex), 1e-8, 10)
    assert info.iterations == 0 and info.status == "converged" and not np.any(x)


def test_fgmres_block_preconditioned_cube16_uses_fewer_applications():
    """Solver variant: one preconditioner application per step instead of
    BiCGSTAB's two; on the cube the total number of applications drops."""
    c = W.cube16()
    g = op.Grid.from_case(c)
    e = physics.plane_wave(g)
    a = krylov.solve(g, e, 1e-6, 1000, c.block_id, c.n_blocks, 1e-3, 500)
    f = krylov.solve(g, e, 1e-6, 1000, c.block_id, c.n_blocks, 1e-3, 500, method="fgmres")
    assert f.info.status == "converged"
    assert len(f.inner_counts) == f.info.iterations
    assert len(f.inner_counts) < len(a.inner_counts)
    assert np.linalg.norm(f.E_tot - a.E_tot) <= 1e-4 * np.linalg.norm(a.E_tot)


# ---- expanded (overlapping) blocks: restricted additive Schwarz
def _dense_ras(g, block_id, n_blocks, overlap, w):
    """y|B_k = (A_{E_k}^{-1} w|E_k)|B_k by dense LU of A restricted to E_k,
    with E_k found by brute force (Chebyshev distance to block k <= overlap,
    inside the scatterer)."""
    Z, idx = op.dense_matrix(g)
    i, j, k = idx
    n = i.size
    ws = op.to_support(g, w, idx)
    bid = block_id[k, j, i]
    y = np.zeros(3 * n, complex)
    for b in range(n_blocks):
        own = np.nonzero(bid == b)[0]
        if own.size == 0:
            continue
        d = np.max(np.abs(np.stack([i[:, None] - i[own][None, :], j[:, None] - j[own][None, :],
                                    k[:, None] - k[own][None, :]])), axis=0).min(axis=1)
        sset = np.nonzero(d <= overlap)[0]
        rows = np.concatenate([sset + c * n for c in range(3)])
        sol = np.linalg.solve(Z[np.ix_(rows, rows)], ws[rows])
        pos = {int(v): q for q, v in enumerate(sset)}
        for c in range(3):
            for v in own:
                y[c * n + v] = sol[c * sset.size + pos[int(v)]]
    return op.from_support(g, y, idx)


@pytest.mark.parametrize("overlap", [1, 2])
def test_expanded_blocks_match_dense_restricted_solves(overlap):
    case, g, e = _problem(56, (4, 5, 6), n_blocks=3)
    rng = np.random.default_rng(1)
    w = (rng.standard_normal((3,) + case.shape) + 1j * rng.standard_normal((3,) + case.shape)) * g.mask
    pre = krylov.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-14, 2000, overlap=overlap)
    y = pre(w)
    want = _dense_ras(g, case.block_id, case.n_blocks, overlap, w)
    assert np.linalg.norm(y - want) <= 1e-10 * np.linalg.norm(want)
    assert np.all(y[:, ~g.mask] == 0)


def test_overlap_zero_is_the_block_diagonal_preconditioner():
    case, g, e = _problem(57, (4, 4, 5), n_blocks=3)
    rng = np.random.default_rng(2)
    w = (rng.standard_normal((3,) + case.shape) + 1j * rng.standard_normal((3,) + case.shape)) * g.mask
    a = krylov.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-12, 500)(w)
    want = _dense_ras(g, case.block_id, case.n_blocks, 0, w)
    assert np.linalg.norm(a - want) <= 1e-9 * np.linalg.norm(want)


def test_overlap_covering_the_scatterer_is_exact():
    """Every expanded block covers the whole scatterer: K2 = A, one outer
    step (the half-step test) gives the dense solution."""
    case, g, e = _problem(58, (3, 4, 4), n_blocks=2)
    s = krylov.solve(g, e, 1e-10, 10, case.block_id, case.n_blocks, 1e-14, 2000, overlap=4)
    assert s.info.iterations == 1
    ref = krylov.solve_dense(g, e)
    assert np.linalg.norm(s.P - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("precondition", [False, True])
def test_cgs_iterates_match_scipy_cgs(precondition):
    """CGS (solver variant): every iterate equals that of an independent
    library implementation of Sonneveld's recurrence with the residual
    recomputed as b - A x (scipy), with and without a right preconditioner."""
    n4 = 4
    kk, jj, ii = np.meshgrid(*[np.arange(n4)] * 3, indexing="ij")
    g = op.Grid(n4, n4, n4, 0.06, 0.06, 0.06, 1.0, np.full((n4,) * 3, 4.0 + 0j))
    block_id = (ii >= 2).astype(np.int32)
    e = physics.plane_wave(g)
    Z, idx = op.dense_matrix(g)
    A = lambda x: op.from_support(g, Z @ op.to_support(g, x, idx), idx)
    b = op.to_support(g, e * g.mask, idx)
    n = b.size
    M_grid = M_s = None
    if precondition:
        i, j, k = idx
        blk = np.tile(block_id[k, j, i], 3)
        Minv = np.linalg.inv(np.where(blk[:, None] == blk[None, :], Z, 0))
        M_grid = lambda w: op.from_support(g, Minv @ op.to_support(g, w, idx), idx)
        M_s = spla.LinearOperator((n, n), matvec=lambda v: Minv @ v, dtype=complex)
    A_s = spla.LinearOperator((n, n), matvec=lambda v: Z @ v, dtype=complex)
    hist = []
    spla.cgs(A_s, b, rtol=1e-30, atol=0.0, maxiter=6, M=M_s, callback=lambda xk: hist.append(xk.copy()))
    assert len(hist) == 6
    for k in range(1, 7):
        x, info = krylov.cgs(A, e * g.mask, 0.0, k, M_grid)
        assert info.iterations == k
        xs = op.to_support(g, x, idx)
        assert np.linalg.norm(xs - hist[k - 1]) <= 1e-12 * np.linalg.norm(hist[k - 1])
        r = op.to_support(g, e * g.mask - A(x), idx)
        assert info.relres == pytest.approx(np.linalg.norm(r) / np.linalg.norm(b), rel=1e-12)


@pytest.mark.parametrize("seed,shape", [(44, (3, 4, 5)), (45, (4, 4, 4))])
def test_cgs_converges_to_dense_lu(seed, shape):
    case, g, e = _problem(seed, shape)
    Pd = krylov.solve_dense(g, e)
    s = krylov.solve(g, e, 1e-12, 3000, method="cgs")
    assert s.info.status == "converged"
    assert np.linalg.norm(s.P - Pd) <= 1e-9 * np.linalg.norm(Pd)
    sp = krylov.solve(g, e, 1e-12, 3000, case.block_id, case.n_blocks, 1e-6, 500, method="cgs")
    assert sp.info.status == "converged"
    assert np.linalg.norm(sp.P - Pd) <= 1e-9 * np.linalg.norm(Pd)
    # two preconditioner applications per step, as in BiCGSTAB
    assert len(sp.inner_counts) == 2 * sp.info.iterations


def test_cgs_exact_preconditioner_one_step_and_zero_rhs():
    A, b = _dense_problem(5)
    Ainv = np.linalg.inv(A)
    x, info = krylov.cgs(lambda v: A @ v, b, 1e-12, 10, precond=lambda w: Ainv @ w)
    assert info.iterations == 1 and info.status == "converged"
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    x, info = krylov.cgs(lambda v: v, np.zeros(4, complex), 1e-8, 10)
    assert info.iterations == 0 and info.status == "converged" and not np.any(x)
