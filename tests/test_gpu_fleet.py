"""vie_solve_many: independent problems of one grid shape solved as one
batch (one launch per step covering every problem's outer system, and one
set of batched inner solves for all their blocks), against the same
problems solved one by one.

* Unpreconditioned: every problem's per-system arithmetic in the batch is
  that of its solve alone (same kernels, same kernel variants, per-system
  reductions), so the fields and step counts are identical bit for bit.
* Block-preconditioned: the batch regroups the blocks of all problems (with
  each problem's own spectra) and runs them on the batched kernels, so its
  rounding differs from the solves alone; the discrete solution is unique,
  and at relative residual 1e-10 in FP64 both are within 1e-8 of each other
  (mixed precision with refinement to 1e-9: 1e-7).
* The sweep's problems (different wavelengths, geometries and partitions on
  one grid shape) in mixed precision: every batched result reaches its
  tolerance and matches its solve alone.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2501_13512_amd import vie as V  # noqa: E402


def _grid(c):
    return V.make_grid(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.wavelength)


def _problems(ctx, cases, blocks):
    return [V.Problem(_grid(c), c.eps, c.block_id if blocks else None, c.n_blocks if blocks else 0, ctx=ctx)
            for c in cases]


def _incident(P, c):
    return torch.from_numpy(V.vie_plane_wave(P.grid, c.kdir, c.pol)).cuda()


def _alone(Ps, cases, opts):
    out = []
    for P, c in zip(Ps, cases):
        e = _incident(P, c)
        y = torch.empty_like(e)
        st = V.vie_stats()
        code = V.vie_solve_device(P.handle, e, opts, y, None, st)
        torch.cuda.synchronize()
        out.append((code, y.cpu().numpy(), st.outer_iters, st.relres_true))
    return out


def _many(Ps, cases, opts):
    es = [_incident(P, c) for P, c in zip(Ps, cases)]
    ys = [torch.empty_like(e) for e in es]
    st = (V.vie_stats * len(Ps))()
    code = V.vie_solve_many([P.handle for P in Ps], es, opts, ys, stats=st)
    torch.cuda.synchronize()
    return code, [y.cpu().numpy() for y in ys], [st[r].outer_iters for r in range(len(Ps))], \
        [st[r].relres_true for r in range(len(Ps))]


def _tiny_set(shape, k0s):
    cases = []
    for i, lam in enumerate(k0s):
        c = W.random_tiny(9100 + i, shape, fill=0.8, n_blocks=3)
        c.wavelength = lam
        c.dx = c.dy = c.dz = 0.05 * lam * (1 + 0.1 * i)   # spacing differs too
        cases.append(c)
    return cases


@pytest.mark.parametrize("prec", [V.VIE_FP64, V.VIE_MIXED])
def test_plain_batch_equals_solves_alone(vie_ctx, prec):
    cases = _tiny_set((7, 9, 11), [1.0, 1.3, 0.8, 1.1])
    Ps = _problems(vie_ctx, cases, blocks=False)
    try:
        opts = V.make_opts(tol_outer=1e-8, precondition=False, precision=prec, maxit_outer=500, max_refine=0)
        alone = _alone(Ps, cases, opts)
        code, ys, its, _ = _many(Ps, cases, opts)
        assert code in (V.VIE_OK, V.VIE_NOT_CONVERGED)
        for r, (c, y, it, _) in enumerate(alone):
            assert it == its[r], (r, it, its[r])
            assert np.array_equal(y, ys[r]), r
    finally:
        for P in Ps:
            P.close()


@pytest.mark.parametrize("prec,tol,bar", [(V.VIE_FP64, 1e-10, 1e-8), (V.VIE_MIXED, 1e-9, 1e-7)])
def test_preconditioned_batch_matches_solves_alone(vie_ctx, prec, tol, bar):
    """Cubes with eight octant blocks each, at different wavelengths and
    permittivities: the blocks of all problems form one group of 8 x 4
    systems with four different spectra."""
    cases = []
    for i, (lam, eps) in enumerate([(1.0, 4.0), (1.2, 2.5), (0.9, 3.0), (1.05, 2.0)]):
        c = W.cube16()
        c.wavelength = lam
        c.eps = np.where(c.eps != 1.0, eps, 1.0).astype(np.complex128)
        cases.append(c)
    Ps = _problems(vie_ctx, cases, blocks=True)
    try:
        opts = V.make_opts(tol_outer=tol, tol_inner=1e-3, precision=prec, maxit_outer=2000, max_refine=5)
        alone = _alone(Ps, cases, opts)
        code, ys, its, rel = _many(Ps, cases, opts)
        assert code == V.VIE_OK
        for r, (c, y, it, rr) in enumerate(alone):
            assert c == V.VIE_OK and rr <= tol and rel[r] <= tol
            assert np.linalg.norm(ys[r] - y) <= bar * np.linalg.norm(y), r
    finally:
        for P in Ps:
            P.close()


def test_sweep_problems_in_one_batch(vie_ctx):
    """Five sweep problems on the 32^3 grid (wavelengths 480-726 nm, four
    pillar or sphere blocks each) in mixed precision with the block
    preconditioner at tolerance 1e-8 (refinement allowed): every result
    reaches it and lies within 1e-6 of its solve alone."""
    bs = [b for b in range(64) if (W.sweep_case(b).nx, W.sweep_case(b).nz) == (32, 32)][:5]
    cases = [W.sweep_case(b) for b in bs]
    Ps = _problems(vie_ctx, cases, blocks=True)
    try:
        opts = V.make_opts(tol_outer=1e-8, tol_inner=1e-2, precision=V.VIE_MIXED, maxit_outer=3000, max_refine=5)
        alone = _alone(Ps, cases, opts)
        code, ys, its, rel = _many(Ps, cases, opts)
        assert code == V.VIE_OK
        for r, (c, y, it, rr) in enumerate(alone):
            assert c == V.VIE_OK and rel[r] <= 1e-8
            assert np.linalg.norm(ys[r] - y) <= 1e-6 * np.linalg.norm(y), r
    finally:
        for P in Ps:
            P.close()


def test_many_rejects_mismatched_shapes_and_duplicates(vie_ctx):
    a = W.random_tiny(9200, (4, 5, 6), fill=0.8, n_blocks=2)
    b = W.random_tiny(9201, (4, 5, 7), fill=0.8, n_blocks=2)
    Ps = _problems(vie_ctx, [a, b], blocks=True)
    try:
        es = [_incident(P, c) for P, c in zip(Ps, [a, b])]
        ys = [torch.empty_like(e) for e in es]
        opts = V.make_opts(tol_outer=1e-6, precision=V.VIE_FP64)
        with pytest.raises(V.VieError):
            V.vie_solve_many([Ps[0].handle, Ps[1].handle], es, opts, ys)
        with pytest.raises(V.VieError):
            V.vie_solve_many([Ps[0].handle, Ps[0].handle], [es[0], es[0]], opts, [ys[0], ys[0]])
        # one problem: its solve alone (unpreconditioned: this random
        # partition interleaves the blocks voxel by voxel)
        po = V.make_opts(tol_outer=1e-8, precondition=False, precision=V.VIE_FP64, maxit_outer=2000)
        st = (V.vie_stats * 1)()
        assert V.vie_solve_many([Ps[0].handle], [es[0]], po, [ys[0]], stats=st) == V.VIE_OK
        alone = torch.empty_like(es[0])
        assert V.vie_solve_device(Ps[0].handle, es[0], po, alone, None, V.vie_stats()) == V.VIE_OK
        torch.cuda.synchronize()
        assert st[0].relres_true <= 1e-8 and torch.equal(ys[0], alone)
    finally:
        for P in Ps:
            P.close()
