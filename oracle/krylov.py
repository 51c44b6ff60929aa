"""BiCGSTAB with the block-diagonal right preconditioner (Sec. II-B).

Test infrastructure (see ``oracle/__init__``).

The outer solve is BiCGSTAB (van der Vorst, ref. [18] of the paper) applied
to the right-preconditioned system A K2^{-1} (K2 x) = b, K1 = I, as the
paper states in Sec. II-B; each iteration needs the two extra solves
y = K2^{-1} p and z = K2^{-1} s.  K2 is the block-diagonal part of A for a
partition of the scatterer into geometric blocks (eq. (10)); every block
matrix A_k keeps all x/y/z couplings (eq. (11)) and is itself solved by
BiCGSTAB with FFT products to a loose ("softened") tolerance.  The block
solutions are written back into one vector for the outer iteration.

Readings where the paper is silent:

* inner products are conjugated in the first argument; the shadow vector is
  the initial residual; x0 = 0 for the outer and for every inner solve;
* stopping uses the recursive residual, ||r|| / ||b|| in the 2-norm, and is
  also tested after the half step (s);
* an inner solve that reaches its iteration cap (or breaks down) returns its
  last iterate; a block whose right-hand side is zero returns zero;
* one "step" is one pass of the loop below.

Solver variants beside the paper's BiCGSTAB: flexible GMRES (``fgmres``)
and conjugate gradient squared (``cgs``), the latter named by the paper as
another applicable Krylov method (Sec. II-B).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg
import scipy.ndimage

from .operator import FFTOperator, Grid, dense_matrix, from_support, to_support


@dataclasses.dataclass
class KrylovInfo:
    iterations: int = 0
    status: str = "not_converged"     # converged | not_converged | breakdown
    relres: float = float("nan")
    history: List[float] = dataclasses.field(default_factory=list)
    half_step: bool = False


def _dot(a, b) -> complex:
    """<a, b> = sum conj(a) b, summed by numpy's pairwise summation in a fixed
    order (a BLAS dot product may split the sum over threads, which makes the
    rounding, and so the iterates, depend on the machine's core count)."""
    return complex(np.sum(np.conj(a.ravel()) * b.ravel()))


def _norm(a) -> float:
    """2-norm with the same fixed-order summation as ``_dot``."""
    v = a.ravel()
    return float(np.sqrt(np.sum(v.real * v.real + v.imag * v.imag)))


def bicgstab(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float,
             maxit: int, precond: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Right-preconditioned BiCGSTAB; returns (x, KrylovInfo).

    With ``precond`` None the preconditioner is the identity.
    """
    M = precond if precond is not None else (lambda w: w)
    x = np.zeros_like(b)
    r = b.copy()
    rhat = r.copy()
    nb = _norm(b)
    info = KrylovInfo()
    if nb == 0.0:
        info.status, info.relres = "converged", 0.0
        return x, info
    rho_old = alpha = omega = 1.0 + 0.0j
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    for it in range(1, maxit + 1):
        info.iterations = it
        rho = _dot(rhat, r)
        if rho == 0:
            info.status = "breakdown"
            break
        if it == 1:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        y = M(p)
        v = apply_A(y)
        den = _dot(rhat, v)
        if den == 0:
            info.status = "breakdown"
            break
        alpha = rho / den
        s = r - alpha * v
        ns = _norm(s) / nb
        if ns <= tol:
            x = x + alpha * y
            info.status, info.relres, info.half_step = "converged", ns, True
            info.history.append(ns)
            return x, info
        z = M(s)
        t = apply_A(z)
        tt = _dot(t, t)
        if tt == 0:
            info.status = "breakdown"
            break
        omega = _dot(t, s) / tt
        x = x + alpha * y + omega * z
        r = s - omega * t
        nr = _norm(r) / nb
        info.history.append(nr)
        info.relres = nr
        if nr <= tol:
            info.status = "converged"
            return x, info
        if omega == 0:
            info.status = "breakdown"
            break
        rho_old = rho
    return x, info


def _givens(a: complex, b: complex):
    """Complex plane rotation (c real, s complex) with [c, s; -conj(s), c]
    (a, b) = (r, 0)."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, complex(np.conj(b) / abs(b))
    d = np.hypot(abs(a), abs(b))
    return abs(a) / d, complex((a / abs(a)) * np.conj(b) / d)


def fgmres(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float, maxit: int,
           restart: int = 30, precond: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Flexible GMRES(restart), right preconditioned (Saad, SIAM J. Sci.
    Comput. 14 (1993)): the preconditioned vectors z_j = M_j(v_j) are kept, so
    the preconditioner may change from step to step (an inner iterative
    solve).  Arnoldi by modified Gram-Schmidt, complex Givens rotations on
    the Hessenberg matrix; the residual norm |g_{j+1}| of the small least-
    squares problem is the stopping test (relative to ||b||).  A step is one
    preconditioner application and one product.  At a restart or at the end
    x += Z y and the residual is recomputed from b - A x."""
    M = precond if precond is not None else (lambda w: w)
    x = np.zeros_like(b)
    nb = _norm(b)
    info = KrylovInfo()
    if nb == 0.0:
        info.status, info.relres = "converged", 0.0
        return x, info
    r = b.copy()
    it = 0
    while True:
        beta = _norm(r)
        info.relres = beta / nb
        if beta / nb <= tol:
            info.status = "converged"
            return x, info
        if it >= maxit:
            return x, info
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        cs, sn = [], []
        k = 0
        done = False
        for j in range(m):
            it += 1
            k = j + 1
            z = M(V[j])
            Z.append(z)
            w = apply_A(z)
            for i in range(j + 1):
                H[i, j] = _dot(V[i], w)
                w = w - H[i, j] * V[i]
            h = _norm(w)
            H[j + 1, j] = h
            for i in range(j):
                a0, a1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a0 + sn[i] * a1
                H[i + 1, j] = -np.conj(sn[i]) * a0 + cs[i] * a1
            c, s_ = _givens(H[j, j], H[j + 1, j])
            cs.append(c)
            sn.append(s_)
            H[j, j] = c * H[j, j] + s_ * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s_) * g[j]
            g[j] = c * g[j]
            res = abs(g[j + 1]) / nb
            info.history.append(res)
            info.iterations = it
            if res <= tol or it >= maxit or h == 0.0:
                done = True
                break
            V.append(w / h)
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - apply_A(x)
        if done and abs(g[k]) / nb <= tol:
            info.relres = _norm(r) / nb
            info.status = "converged"
            return x, info
        if it >= maxit:
            info.relres = _norm(r) / nb
            return x, info


@dataclasses.dataclass
class _Block:
    index: int
    sl: tuple                  # slices (z, y, x) of the bounding box of the solve set
    member: np.ndarray         # bool [bz, by, bx]: the voxels solved for
    op: FFTOperator
    own: np.ndarray            # bool [bz, by, bx]: the block's own voxels (kept)


def cgs(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float, maxit: int,
        precond: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Conjugate gradient squared (Sonneveld, SIAM J. Sci. Stat. Comput. 10
    (1989)), right preconditioned, x0 = 0: one of the Krylov solvers the
    paper lists as applicable (Sec. II-B).  The residual is recomputed as
    b - A x after every step (the form of the standard template that
    replaces the recursive update; same two products per step).  A step is
    two preconditioner applications and two products; the stopping test is
    ||b - A x|| / ||b|| after the step."""
    M = precond if precond is not None else (lambda w: w)
    x = np.zeros_like(b)
    nb = _norm(b)
    info = KrylovInfo()
    if nb == 0.0:
        info.status, info.relres = "converged", 0.0
        return x, info
    r = b.copy()
    rhat = r.copy()
    rho = _dot(rhat, r)
    u = p = q = None
    for it in range(1, maxit + 1):
        if it == 1:
            u = r.copy()
            p = r.copy()
        else:
            rho_new = _dot(rhat, r)
            if rho_new == 0.0:
                info.status = "breakdown"
                return x, info
            beta = rho_new / rho
            rho = rho_new
            u = r + beta * q
            p = u + beta * (q + beta * p)
        v = apply_A(M(p))
        rv = _dot(rhat, v)
        if rv == 0.0:
            info.status = "breakdown"
            return x, info
        alpha = rho / rv
        q = u - alpha * v
        x = x + alpha * M(u + q)
        r = b - apply_A(x)
        info.iterations = it
        info.relres = _norm(r) / nb
        info.history.append(info.relres)
        if info.relres <= tol:
            info.status = "converged"
            return x, info
    return x, info


def expanded_block(grid: Grid, block_id: np.ndarray, k: int, overlap: int) -> np.ndarray:
    """Scatterer voxels within ``overlap`` voxels of block k in every axis
    (the block dilated by a (2 overlap + 1)^3 cube, restricted to S)."""
    own = block_id == k
    if overlap <= 0:
        return own
    grown = scipy.ndimage.binary_dilation(own, structure=np.ones((3, 3, 3), dtype=bool), iterations=overlap)
    return grown & grid.mask


class BlockPreconditioner:
    """y = K2^{-1} w with K2 = blockdiag(A_1, ..., A_N) (eq. (10)).

    Block k is the set of voxels with ``block_id == k``.  Its matrix A_k is
    A restricted to those voxels, applied with the FFT product on the block's
    bounding box with every other voxel masked as vacuum.

    ``overlap`` > 0 expands every block (the paper names expanded blocks as
    future work): block k is solved on E_k, its voxels dilated by ``overlap``
    voxels in every axis within the scatterer, and only its own voxels are
    kept (restricted additive Schwarz: y|B_k = (A_{E_k}^{-1} w|E_k)|B_k).
    With overlap 0 this is the block-diagonal preconditioner above.
    """

    def __init__(self, grid: Grid, block_id: np.ndarray, n_blocks: int, tol: float, maxit: int, pad: int = 0,
                 product: str = "fp64", overlap: int = 0):
        self.tol = tol
        self.maxit = maxit
        self.blocks: List[_Block] = []
        self.inner_counts: List[List[int]] = []
        for k in range(n_blocks):
            if not np.any(block_id == k):
                continue
            solve_set = expanded_block(grid, block_id, k, overlap)
            kk, jj, ii = np.nonzero(solve_set)
            sl = (slice(kk.min(), kk.max() + 1), slice(jj.min(), jj.max() + 1),
                  slice(ii.min(), ii.max() + 1))
            member = solve_set[sl]
            own = block_id[sl] == k
            sub_eps = np.where(member, grid.eps[sl], 1.0 + 0.0j)
            sub = Grid(sub_eps.shape[2], sub_eps.shape[1], sub_eps.shape[0],
                       grid.dx, grid.dy, grid.dz, grid.wavelength, sub_eps)
            self.blocks.append(_Block(k, sl, member, FFTOperator(sub, pad, product), own))

    def __call__(self, w: np.ndarray) -> np.ndarray:
        y = np.zeros_like(w)
        counts = []
        for blk in self.blocks:
            bk = w[(slice(None),) + blk.sl] * blk.member
            if _norm(bk) == 0.0:
                counts.append(0)
                continue
            yk, info = bicgstab(blk.op, bk, self.tol, self.maxit)
            y[(slice(None),) + blk.sl] += yk * blk.own
            counts.append(info.iterations)
        self.inner_counts.append(counts)
        return y


@dataclasses.dataclass
class Solution:
    P: np.ndarray              # [3, nz, ny, nx], P = J / (j omega eps0)
    E_tot: np.ndarray          # P / chi on S, 0 in vacuum (eq. (2))
    info: KrylovInfo
    inner_counts: List[List[int]]
    # mixed mode only (``solve_mixed``): FP64 true residual at the end, the
    # number of correction solves and their total outer steps, and the true
    # residual after the main loop and after every correction
    relres_true: float = float("nan")
    refine_steps: int = 0
    refine_iters: int = 0
    true_history: List[float] = dataclasses.field(default_factory=list)


def masked_rhs(grid: Grid, e_inc: np.ndarray) -> np.ndarray:
    return e_inc * grid.mask


def total_field(grid: Grid, P: np.ndarray) -> np.ndarray:
    return P * grid.chi_inv


def solve(grid: Grid, e_inc: np.ndarray, tol_outer: float, maxit_outer: int = 1000,
          block_id: Optional[np.ndarray] = None, n_blocks: int = 0,
          tol_inner: float = 1e-2, maxit_inner: int = 500, pad: int = 0, product: str = "fp64",
          method: str = "bicgstab", restart: int = 30, overlap: int = 0) -> Solution:
    """Solve A P = E_inc on S; block preconditioner if ``block_id`` is given.

    ``pad`` lengthens every circulant embedding (same operator, different
    rounding); comparing runs with pad 0 and pad > 0 measures how much
    rounding alone moves the iterates at a given tolerance.
    ``product="c64"`` runs every FFT convolution in complex64 (the mixed
    mode's products); vectors and inner products stay FP64.
    ``method="fgmres"`` replaces the outer BiCGSTAB by flexible GMRES(restart),
    ``method="cgs"`` by conjugate gradient squared (solver variants; the
    paper's method is BiCGSTAB)."""
    A = FFTOperator(grid, pad, product)
    b = masked_rhs(grid, e_inc)
    pre = None
    if block_id is not None:
        pre = BlockPreconditioner(grid, block_id, n_blocks, tol_inner, maxit_inner, pad, product, overlap)
    if method == "fgmres":
        P, info = fgmres(A, b, tol_outer, maxit_outer, restart, pre)
    elif method == "cgs":
        P, info = cgs(A, b, tol_outer, maxit_outer, pre)
    else:
        P, info = bicgstab(A, b, tol_outer, maxit_outer, pre)
    return Solution(P, total_field(grid, P), info, pre.inner_counts if pre is not None else [])


def solve_dense(grid: Grid, e_inc: np.ndarray) -> np.ndarray:
    """Reference solution of A P = E_inc by dense LU (tiny grids only)."""
    Z, idx = dense_matrix(grid)
    b = to_support(grid, masked_rhs(grid, e_inc), idx)
    x = scipy.linalg.solve(Z, b)
    return from_support(grid, x, idx)


def solve_mixed(grid: Grid, e_inc: np.ndarray, tol_outer: float, maxit_outer: int = 1000,
                block_id: Optional[np.ndarray] = None, n_blocks: int = 0, tol_inner: float = 1e-2,
                maxit_inner: int = 500, max_refine: int = 3, pad: int = 0) -> Solution:
    """Mixed precision with iterative refinement (the precision change on top
    of the paper's method; the paper states no precision).

    1. The main loop is the BiCGSTAB of ``solve`` with every operator product
       (outer and inside the block solves) in complex64; vectors, inner
       products and norms stay FP64.
    2. Its iterate x is checked with the FP64 product: r = b - A x.
    3. While ||r|| / ||b|| > tol_outer and fewer than ``max_refine``
       corrections were made: solve A d = r with the same mixed loop, x += d,
       and form r again in FP64.  A correction is stopped once it has brought
       the residual to the outer tolerance relative to ||b||, i.e. at
       ||r - A d|| <= (tol_outer / relres) ||r||, but never looser than
       halving it (tolerance min(0.5, tol_outer / relres)).
    4. The step count of the main loop is the one compared between
       implementations; the corrections are counted separately.

    A main loop that breaks down is not refined.
    """
    A64 = FFTOperator(grid, pad, "fp64")
    A32 = FFTOperator(grid, pad, "c64")
    b = masked_rhs(grid, e_inc)
    nb = _norm(b)
    pre = None
    if block_id is not None:
        pre = BlockPreconditioner(grid, block_id, n_blocks, tol_inner, maxit_inner, pad, "c64")
    x, info = bicgstab(A32, b, tol_outer, maxit_outer, pre)
    r = b - A64(x)
    rel = _norm(r) / nb if nb > 0 else 0.0
    hist = [rel]
    refine = refine_iters = 0
    while info.status != "breakdown" and nb > 0 and rel > tol_outer and refine < max_refine:
        tol_c = min(0.5, tol_outer / rel)
        d, ic = bicgstab(A32, r, tol_c, maxit_outer, pre)
        x = x + d
        refine += 1
        refine_iters += ic.iterations
        r = b - A64(x)
        rel = _norm(r) / nb
        hist.append(rel)
    return Solution(x, total_field(grid, x), info, pre.inner_counts if pre is not None else [],
                    relres_true=rel, refine_steps=refine, refine_iters=refine_iters, true_history=hist)
