"""GPU parity of the rooftop discretisation (Sec. II-A, eq. (5); the split
of eqs. (7)-(9)) against the oracle's rooftop operator, element by element:
products on random padded grids (plane-kernel and row-kernel shapes, short
and long z columns, ragged sizes, every z-pass variant), the padded
metasurface at full size, plain solves of a dielectric sphere, and the
argument checks of the rooftop entry points.

Products: max |GPU - oracle| / max |oracle| <= 1e-12 in FP64 and <= 1e-5
in mixed mode (complex FP32 FFT), as for the collocated product; faces
without an unknown are exactly zero.  Solves: the GPU and the oracle run
BiCGSTAB to the same tolerance from x0 = 0; the solutions agree to a few
times tol times the conditioning (bars stated per test)."""
import numpy as np
import pytest

import workloads as W
from oracle import rooftop as rt, operator as op, physics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2501_13512_amd import vie as V  # noqa: E402

TOL = {V.VIE_FP64: 1e-12, V.VIE_MIXED: 1e-5}

# interior shapes (nz, ny, nx); the grids are one vacuum layer larger per side
SMALL = [(1, 1, 1), (2, 1, 3), (3, 5, 4), (6, 5, 4), (4, 7, 2)]
MID = [(16, 16, 16), (12, 20, 33), (7, 48, 24), (40, 21, 13), (30, 14, 14), (9, 3, 100), (32, 64, 64),
       # lengths 36 (z only), 72, 144 and 288
       (16, 33, 9), (24, 7, 68), (32, 10, 128)]


def _case(seed, interior, fill=0.7):
    return W.padded(W.random_tiny(seed, interior, fill=fill))


def _grid(case):
    return V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.wavelength)


def _rand(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)


def _matvec(P, x, prec):
    xd = torch.from_numpy(x).cuda()
    yd = torch.full_like(xd, complex("nan"))
    V.vie_matvec(P.handle, prec, xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _assert_close(got, want, fmask, tol):
    assert np.all(got[~fmask] == 0), "faces without an unknown must be zero"
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= tol, err


def _check_product(ctx, case, seed, precs=(V.VIE_FP64, V.VIE_MIXED), variants=(None,)):
    g = op.Grid.from_case(case)
    fm = rt.face_mask(g)
    x = _rand(seed, case.shape)
    want = rt.RooftopFFT(g)(x)
    P = V.Problem(_grid(case), case.eps, ctx=ctx, rooftop=True)
    try:
        for prec in precs:
            for v in variants:
                if v is not None:
                    V.vie_problem_set_zpass(P.handle, prec, v)
                print(f"rooftop product {case.name} prec {prec} variant {v}", flush=True)
                _assert_close(_matvec(P, x, prec), want, fm, TOL[prec])
    finally:
        P.close()


@pytest.mark.parametrize("interior", SMALL)
def test_rooftop_product_small(vie_ctx, interior):
    seed = 5000 + sum(s * 31 ** i for i, s in enumerate(interior))
    _check_product(vie_ctx, _case(seed, interior), seed)


@pytest.mark.parametrize("interior", MID)
def test_rooftop_product_ragged(vie_ctx, interior):
    seed = 6000 + sum(s * 31 ** i for i, s in enumerate(interior))
    _check_product(vie_ctx, _case(seed, interior, fill=0.6), seed)


def test_rooftop_zpass_variants(vie_ctx):
    """Every column-set z-pass variant (long columns: lz = 64 and 96) gives
    the oracle's product; the mirror-column variant is refused."""
    for interior in [(30, 14, 14), (40, 21, 13)]:
        seed = 7000 + sum(interior)
        _check_product(vie_ctx, _case(seed, interior, fill=0.6), seed, variants=(0, 2, 3, 4))
    case = _case(1, (3, 3, 3))
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        with pytest.raises(V.VieError) as e:
            V.vie_problem_set_zpass(P.handle, V.VIE_FP64, 1)
        assert e.value.code == V.VIE_EINVAL
        assert P.info().zpass_variant[0] != 1 and P.info().zpass_tune_ms[0][1] == -1
    finally:
        P.close()


def test_rooftop_product_padded_metasurface_full_size(vie_ctx):
    """The metasurface (8 x 8 pillars on a slab, 128 x 128 x 32 at lambda/40)
    with one vacuum layer per side, 130 x 130 x 34: every face, both
    precisions, in the launch configuration the product uses there."""
    _check_product(vie_ctx, W.padded(W.metasurface()), 11)


def test_rooftop_face_contrast_cases(vie_ctx):
    """Faces whose mean of 1/eps is 1 (eps 2 next to eps 2/3) and faces
    between vacuum cells carry no unknown; an all-vacuum grid gives 0."""
    eps = np.ones((5, 5, 6), complex)
    eps[2, 2, 2], eps[2, 2, 3] = 2.0, 2.0 / 3.0
    eps[2, 1, 2] = 4.0 - 1.0j
    case = W.Case("contrast", 6, 5, 5, 0.05, 0.05, 0.05, 1.0, eps, np.full(eps.shape, -1, np.int32), 0, 1e-8, 1e-2)
    g = op.Grid.from_case(case)
    fm = rt.face_mask(g)
    assert not fm[0, 2, 2, 2]            # the m = 1 face
    _check_product(vie_ctx, case, 3)
    vac = W.Case("vacuum", 4, 4, 4, 0.1, 0.1, 0.1, 1.0, np.ones((4, 4, 4), complex),
                 np.full((4, 4, 4), -1, np.int32), 0, 1e-8, 1e-2)
    P = V.Problem(_grid(vac), vac.eps, ctx=vie_ctx, rooftop=True)
    try:
        assert np.all(_matvec(P, _rand(4, vac.shape), V.VIE_FP64) == 0)
    finally:
        P.close()


def test_rooftop_argument_checks(vie_ctx):
    """Non-vacuum boundary layers, preconditioning without blocks and
    batches mixing rooftop and collocated problems are refused with
    VIE_EINVAL."""
    case = W.random_tiny(9, (4, 4, 4), fill=1.0)
    with pytest.raises(V.VieError) as e:
        V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    assert e.value.code == V.VIE_EINVAL and "vacuum" in str(e.value)
    case = _case(9, (4, 4, 4))
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        n = 3 * case.nvox
        x = torch.zeros(n, dtype=torch.complex128, device="cuda")
        y = torch.zeros_like(x)
        st = V.vie_stats()
        with pytest.raises(V.VieError) as e:
            V.vie_solve_device(P.handle, x, V.make_opts(precondition=True), y, None, st)
        assert e.value.code == V.VIE_EINVAL
        cc = W.random_tiny(9, (6, 6, 6), fill=0.5)
        C = V.Problem(_grid(cc), cc.eps, ctx=vie_ctx)
        try:
            with pytest.raises(V.VieError) as e:
                V.vie_solve_many([P.handle, C.handle], [x, x], V.make_opts(precondition=False), [y, y])
            assert e.value.code == V.VIE_EINVAL
        finally:
            C.close()
    finally:
        P.close()


@pytest.mark.parametrize("prec,tol", [(V.VIE_FP64, 1e-12), (V.VIE_MIXED, 1e-5)])
def test_rooftop_total_field_box_matches_oracle(vie_ctx, prec, tol):
    """E_inc + T P at every face centre of the box, vacuum faces included,
    except the faces of the last cell layer along their own axis (their
    second cell is outside the grid; 0 on output)."""
    case = _case(71, (5, 6, 4), fill=0.7)
    g = op.Grid.from_case(case)
    fm = rt.face_mask(g)
    Pf = _rand(72, case.shape) * fm
    e = rt.plane_wave(g, (0.6, 0.0, 0.8), (0.8, 0.0, -0.6))
    want = e + rt.RooftopFFT(g).scatter(Pf)
    want[0, :, :, -1] = 0
    want[1, :, -1, :] = 0
    want[2, -1, :, :] = 0
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        out = torch.full((3,) + case.shape, complex("nan"), dtype=torch.complex128, device="cuda")
        V.vie_total_field_box(P.handle, prec, torch.from_numpy(Pf).cuda(), torch.from_numpy(e).cuda(), out)
        got = out.cpu().numpy()
    finally:
        P.close()
    assert np.abs(got - want).max() / np.abs(want).max() <= tol


@pytest.mark.parametrize("prec", [V.VIE_FP64, V.VIE_MIXED])
def test_rooftop_plain_batch_equals_separate_solves(vie_ctx, prec):
    """Three incident waves as one plain batch: bitwise the solves one by
    one, and each at the oracle's solution."""
    case = _sphere()
    g = op.Grid.from_case(case)
    waves = [((0.0, 0.0, 1.0), (1.0, 0.0, 0.0)), ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
             ((0.6, 0.0, 0.8), (0.8, 0.0, -0.6))]
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        e = torch.from_numpy(np.stack([V.vie_plane_wave_faces(P.grid, k, p) for k, p in waves])).cuda()
        opts = V.make_opts(tol_outer=1e-10, precondition=False, precision=prec, maxit_outer=2000)
        want, iters = [], []
        for r in range(3):
            out = torch.empty_like(e[r])
            pol = torch.empty_like(e[r])
            st = V.vie_stats()
            V.vie_solve_device(P.handle, e[r].contiguous(), opts, out, pol, st)
            torch.cuda.synchronize()
            want.append(pol.cpu().numpy())
            iters.append(st.outer_iters)
        out = torch.empty_like(e)
        pol = torch.empty_like(e)
        stats = (V.vie_stats * 3)()
        assert V.vie_solve_batch(P.handle, 3, e, opts, out, pol, stats) == V.VIE_OK
        torch.cuda.synchronize()
        got = pol.cpu().numpy()
    finally:
        P.close()
    assert [stats[r].outer_iters for r in range(3)] == iters
    assert np.array_equal(got, np.stack(want))
    for r, (k, p) in enumerate(waves):
        ref, info = rt.solve(g, rt.plane_wave(g, k, p), 1e-12, 3000)
        assert np.abs(got[r] - ref).max() <= 1e-7 * np.abs(ref).max()


def _sphere():
    return W.sphere(6, 30.0, 2.25, pad=1)      # 14^3 grid, k a = 2 pi / 5


@pytest.mark.parametrize("prec,tol,bar", [(V.VIE_FP64, 1e-10, 1e-8), (V.VIE_MIXED, 1e-9, 1e-7)])
def test_rooftop_sphere_solve_matches_oracle(vie_ctx, prec, tol, bar):
    """Plain BiCGSTAB solve of the voxelised sphere (eps 2.25, radius 6 cells)
    under x-polarised incidence along z: the GPU's face-centred plane wave
    equals the oracle's, and the solution P and the face field P / chi_f
    agree with the oracle's solve to `bar` (relative, max norm)."""
    case = _sphere()
    g = op.Grid.from_case(case)
    e_or = rt.plane_wave(g)
    e_gpu = V.vie_plane_wave_faces(_grid(case), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0))
    assert np.abs(e_gpu - e_or).max() <= 1e-13
    P_or, info = rt.solve(g, e_or, 1e-12, 5000)
    assert info.status == "converged"
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        ed = torch.from_numpy(e_gpu).cuda()
        et = torch.zeros_like(ed)
        pol = torch.zeros_like(ed)
        st = V.vie_stats()
        opts = V.make_opts(tol_outer=tol, maxit_outer=2000, precondition=False, precision=prec)
        code = V.vie_solve_device(P.handle, ed, opts, et, pol, st)
        torch.cuda.synchronize()
        print(f"rooftop sphere solve prec {prec}: {st.outer_iters} steps, relres {st.relres_true:.2e}", flush=True)
        assert code == V.VIE_OK and st.relres_true <= 2 * tol
        Pg = pol.cpu().numpy()
        fm = rt.face_mask(g)
        assert np.all(Pg[~fm] == 0)
        err = np.abs(Pg - P_or).max() / np.abs(P_or).max()
        assert err <= bar, err
        E_or = P_or * rt.face_chi_inv(g)
        Eg = et.cpu().numpy()
        assert np.abs(Eg - E_or).max() / np.abs(E_or).max() <= bar
    finally:
        P.close()


def test_rooftop_far_field_matches_oracle(vie_ctx):
    """Far field of random face unknowns on a non-cubic grid, each radiating
    from its face centre, against the oracle's quadrature."""
    case = _case(96, (4, 6, 5), fill=0.8)
    case.dx, case.dy, case.dz = 0.04, 0.05, 0.03
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(97)
    Pf = _rand(98, case.shape) * rt.face_mask(g)
    d = rng.standard_normal((29, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    want = rt.far_field_vector(g, Pf, d)
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        got = V.vie_far_field(P.handle, torch.from_numpy(Pf).cuda(), d)
    finally:
        P.close()
    assert np.abs(got - want).max() / np.abs(want).max() <= 1e-11


@pytest.mark.parametrize("eps,r,tol_rcs", [(2.25, 8, 0.03), (-1.05 - 5.62j, 12, 0.04)])
def test_rooftop_mie_comparison_on_gpu(vie_ctx, eps, r, tol_rcs):
    """The whole rooftop path on the GPU against the Mie series: a voxelised
    sphere (k a = 2 pi / 5, one vacuum layer per side) solved in FP64 without
    preconditioner, E-plane RCS from the GPU far field; the bars are the
    oracle's own (the discretisation error, not the kernels', dominates)."""
    lam = r * 40 / 8
    case = W.sphere(r, lam, eps, pad=1)
    g = op.Grid.from_case(case)
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        e = torch.from_numpy(V.vie_plane_wave_faces(P.grid, case.kdir, case.pol)).cuda()
        out = torch.empty_like(e)
        pol = torch.empty_like(e)
        st = V.vie_stats()
        o = V.make_opts(tol_outer=1e-9, maxit_outer=5000, precondition=False, precision=V.VIE_FP64)
        assert V.vie_solve_device(P.handle, e, o, out, pol, st) == V.VIE_OK
        th = np.radians(np.arange(0, 181))
        rh = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=-1)
        sigma = V.vie_rcs(P.handle, pol, rh)
        Pn = pol.cpu().numpy()
    finally:
        P.close()
    print(f"rooftop Mie eps {eps} r {r}: {st.outer_iters} steps", flush=True)
    assert np.linalg.norm(sigma - rt.rcs_eplane(g, Pn, th)) / np.linalg.norm(sigma) <= 1e-10
    mie = physics.mie_rcs_eplane(eps, r, lam, th)
    assert np.linalg.norm(sigma - mie) / np.linalg.norm(mie) <= tol_rcs


# ---------------------------------------------------------------- blocks (eq. (10))
def _blocked_cases():
    return [W.padded(W.random_tiny(41, (4, 5, 6), fill=0.8, n_blocks=3)),
            W.padded(W.mixed_partition(0))]


def _owner(case):
    return rt.face_owner(op.Grid.from_case(case), case.block_id)


@pytest.mark.parametrize("which", [0, 1])
def test_rooftop_block_matvec_matches_oracle(vie_ctx, which):
    """K2 x (every block's matrix on the faces it owns) against the oracle's
    block product, both precisions; the second case has two block box shapes
    (two batched groups)."""
    case = _blocked_cases()[which]
    g = op.Grid.from_case(case)
    M = rt.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-13, 500)
    x = _rand(42 + which, case.shape) * rt.face_mask(g)
    want = M.block_matvec(x)
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        assert P.info().n_block_solver_groups == 0
        for prec in (V.VIE_FP64, V.VIE_MIXED):
            xd = torch.from_numpy(x).cuda()
            yd = torch.full_like(xd, complex("nan"))
            V.vie_block_matvec(P.handle, prec, xd, yd)
            _assert_close(yd.cpu().numpy(), want, rt.face_mask(g), TOL[prec])
    finally:
        P.close()


@pytest.mark.parametrize("which", [0, 1])
def test_rooftop_precond_apply_matches_oracle(vie_ctx, which):
    """K2^{-1} w with tight inner solves: every block's system solved to
    1e-12 on the GPU (FP64) against the oracle's at 1e-13 (both at the exact
    block solutions, so the bar is set by conditioning, 1e-9)."""
    case = _blocked_cases()[which]
    g = op.Grid.from_case(case)
    M = rt.BlockPreconditioner(g, case.block_id, case.n_blocks, 1e-13, 1000)
    w = _rand(52 + which, case.shape) * rt.face_mask(g)
    want = M(w)
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        wd = torch.from_numpy(w).cuda()
        yd = torch.full_like(wd, complex("nan"))
        V.vie_precond_apply(P.handle, V.VIE_FP64, 1e-12, 1000, wd, yd)
        got = yd.cpu().numpy()
    finally:
        P.close()
    _assert_close(got, want, rt.face_mask(g), 1e-9)


@pytest.mark.parametrize("prec,tol,bar", [(V.VIE_FP64, 1e-10, 1e-8), (V.VIE_MIXED, 1e-9, 1e-7)])
def test_rooftop_preconditioned_solve_matches_oracle(vie_ctx, prec, tol, bar):
    """Block-preconditioned BiCGSTAB (inner tol 1e-3) on the two-shape
    partition: the GPU solution equals the oracle's plain solve at 1e-12 (the
    solution is unique; the inexact inner solves only change the path) and
    the GPU needs fewer outer steps than the oracle's plain solve."""
    case = W.padded(W.mixed_partition(0))
    g = op.Grid.from_case(case)
    e = rt.plane_wave(g)
    P0, i0 = rt.solve(g, e, 1e-12, 3000)
    assert i0.status == "converged"
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        ed = torch.from_numpy(V.vie_plane_wave_faces(P.grid, case.kdir, case.pol)).cuda()
        et = torch.empty_like(ed)
        pol = torch.empty_like(ed)
        st = V.vie_stats()
        o = V.make_opts(tol_outer=tol, tol_inner=1e-3, maxit_outer=500, precondition=True, precision=prec)
        assert V.vie_solve_device(P.handle, ed, o, et, pol, st) == V.VIE_OK
        print(f"rooftop preconditioned solve prec {prec}: {st.outer_iters} steps (plain oracle {i0.iterations}), "
              f"inner {st.inner_iters_total}", flush=True)
        Pg = pol.cpu().numpy()
    finally:
        P.close()
    assert np.abs(Pg - P0).max() <= bar * np.abs(P0).max()
    assert st.outer_iters < i0.iterations


def test_rooftop_padded_metasurface_blocks_full_size(vie_ctx):
    """The padded metasurface with its 64 pillar blocks and the slab block:
    K2 x for x on one pillar's faces and on the slab's faces equals the
    oracle's full-grid product masked to that block; then a mixed
    block-preconditioned solve (outer 2e-6, inner 1e-2) whose solution the
    oracle's own product checks (||b - A P|| / ||b||, FP64)."""
    case = W.padded(W.metasurface())
    g = op.Grid.from_case(case)
    owner = _owner(case)
    A = rt.RooftopFFT(g)
    x = _rand(61, case.shape)
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        for k in (0, 27, 64):
            xk = x * (owner == k)
            want = (owner == k) * A(xk)
            xd = torch.from_numpy(xk).cuda()
            yd = torch.full_like(xd, complex("nan"))
            V.vie_block_matvec(P.handle, V.VIE_FP64, xd, yd)
            print(f"padded metasurface block {k}: K2 x", flush=True)
            _assert_close(yd.cpu().numpy(), want, rt.face_mask(g), 1e-12)
        e = V.vie_plane_wave_faces(P.grid, case.kdir, case.pol)
        ed = torch.from_numpy(e).cuda()
        et = torch.empty_like(ed)
        pol = torch.empty_like(ed)
        st = V.vie_stats()
        o = V.make_opts(tol_outer=2e-6, tol_inner=1e-2, maxit_outer=1000, precondition=True,
                        precision=V.VIE_MIXED)
        assert V.vie_solve_device(P.handle, ed, o, et, pol, st) == V.VIE_OK
        print(f"padded metasurface preconditioned mixed solve: {st.outer_iters} steps, "
              f"relres_true {st.relres_true:.2e}", flush=True)
        Pg = pol.cpu().numpy()
    finally:
        P.close()
    b = np.where(rt.face_mask(g), e, 0)
    res = np.linalg.norm(b - A(Pg)) / np.linalg.norm(b)
    assert res <= 3e-6, res


@pytest.mark.parametrize("prec", [V.VIE_FP64, V.VIE_MIXED])
def test_rooftop_problems_in_one_batch(vie_ctx, prec):
    """Three rooftop problems of one grid shape (different permittivities and
    spacings) as one plain vie_solve_many batch: bitwise the solves alone,
    each at the oracle's solution."""
    cases = [_case(80 + i, (6, 6, 6), fill=0.6) for i in range(3)]
    probs = [V.Problem(_grid(c), c.eps, ctx=vie_ctx, rooftop=True) for c in cases]
    try:
        es = [torch.from_numpy(V.vie_plane_wave_faces(p.grid, (0.0, 0.0, 1.0), (1.0, 0.0, 0.0))).cuda()
              for p in probs]
        opts = V.make_opts(tol_outer=1e-10, precondition=False, precision=prec, maxit_outer=2000)
        want, iters = [], []
        for p, e in zip(probs, es):
            out, pol, st = torch.empty_like(e), torch.empty_like(e), V.vie_stats()
            V.vie_solve_device(p.handle, e, opts, out, pol, st)
            torch.cuda.synchronize()
            want.append(pol.cpu().numpy())
            iters.append(st.outer_iters)
        outs = [torch.empty_like(e) for e in es]
        pols = [torch.empty_like(e) for e in es]
        stats = (V.vie_stats * 3)()
        assert V.vie_solve_many([p.handle for p in probs], es, opts, outs, pols, stats) == V.VIE_OK
        torch.cuda.synchronize()
        got = [q.cpu().numpy() for q in pols]
    finally:
        for p in probs:
            p.close()
    assert [stats[r].outer_iters for r in range(3)] == iters
    for r, c in enumerate(cases):
        assert np.array_equal(got[r], want[r]), r
        g = op.Grid.from_case(c)
        ref, _ = rt.solve(g, rt.plane_wave(g), 1e-12, 3000)
        assert np.abs(got[r] - ref).max() <= 1e-7 * np.abs(ref).max()


@pytest.mark.parametrize("solver,prec", [(V.VIE_SOLVER_FGMRES, V.VIE_FP64), (V.VIE_SOLVER_CGS, V.VIE_FP64),
                                         (V.VIE_SOLVER_BICGSTAB, V.VIE_MIXED_INNER)])
def test_rooftop_solver_variants_reach_the_oracle_solution(vie_ctx, solver, prec):
    """Flexible GMRES(30), CGS and BiCGSTAB with FP32 inner solves, all with
    the rooftop block preconditioner on the two-shape partition: each
    solution equals the oracle's (unique) solution within 1e-8."""
    case = W.padded(W.mixed_partition(0))
    g = op.Grid.from_case(case)
    P0, i0 = rt.solve(g, rt.plane_wave(g), 1e-12, 3000)
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        ed = torch.from_numpy(V.vie_plane_wave_faces(P.grid, case.kdir, case.pol)).cuda()
        et, pol, st = torch.empty_like(ed), torch.empty_like(ed), V.vie_stats()
        o = V.make_opts(tol_outer=1e-10, tol_inner=1e-3, maxit_outer=500, precondition=True, precision=prec,
                        solver=solver, restart=30)
        assert V.vie_solve_device(P.handle, ed, o, et, pol, st) == V.VIE_OK
        print(f"rooftop solver {solver} prec {prec}: {st.outer_iters} steps", flush=True)
        Pg = pol.cpu().numpy()
    finally:
        P.close()
    assert np.abs(Pg - P0).max() <= 1e-8 * np.abs(P0).max()


@pytest.mark.parametrize("prec,tol,bar", [(V.VIE_FP64, 1e-10, 1e-8), (V.VIE_MIXED, 1e-9, 1e-7)])
def test_rooftop_preconditioned_batch_of_waves(vie_ctx, prec, tol, bar):
    """Two incident waves as one block-preconditioned batch (the blocks of
    both solved together on the stacked replica): each solution at the
    oracle's."""
    case = W.padded(W.mixed_partition(0))
    g = op.Grid.from_case(case)
    waves = [((0.0, 0.0, 1.0), (1.0, 0.0, 0.0)), ((0.6, 0.0, 0.8), (0.8, 0.0, -0.6))]
    P = V.Problem(_grid(case), case.eps, case.block_id, case.n_blocks, ctx=vie_ctx, rooftop=True)
    try:
        e = torch.from_numpy(np.stack([V.vie_plane_wave_faces(P.grid, k, p) for k, p in waves])).cuda()
        out, pol, stats = torch.empty_like(e), torch.empty_like(e), (V.vie_stats * 2)()
        o = V.make_opts(tol_outer=tol, tol_inner=1e-3, maxit_outer=500, precondition=True, precision=prec)
        assert V.vie_solve_batch(P.handle, 2, e, o, out, pol, stats) == V.VIE_OK
        torch.cuda.synchronize()
        got = pol.cpu().numpy()
    finally:
        P.close()
    for r, (k, p) in enumerate(waves):
        ref, _ = rt.solve(g, rt.plane_wave(g, k, p), 1e-12, 3000)
        assert np.abs(got[r] - ref).max() <= bar * np.abs(ref).max(), r
        assert stats[r].precond_applies > 0


def test_rooftop_preconditioned_problems_in_one_batch(vie_ctx):
    """Three rooftop problems with blocks (different spacings: per-system
    spectra) as one block-preconditioned vie_solve_many batch, FP64: each
    solution at the oracle's."""
    cases = [W.padded(W.random_tiny(90 + i, (5, 6, 6), fill=0.7, n_blocks=3)) for i in range(3)]
    probs = [V.Problem(_grid(c), c.eps, c.block_id, c.n_blocks, ctx=vie_ctx, rooftop=True) for c in cases]
    try:
        es = [torch.from_numpy(V.vie_plane_wave_faces(p.grid, (0.0, 0.0, 1.0), (1.0, 0.0, 0.0))).cuda()
              for p in probs]
        outs = [torch.empty_like(e) for e in es]
        pols = [torch.empty_like(e) for e in es]
        stats = (V.vie_stats * 3)()
        o = V.make_opts(tol_outer=1e-10, tol_inner=1e-3, maxit_outer=500, precondition=True, precision=V.VIE_FP64)
        assert V.vie_solve_many([p.handle for p in probs], es, o, outs, pols, stats) == V.VIE_OK
        torch.cuda.synchronize()
        got = [q.cpu().numpy() for q in pols]
    finally:
        for p in probs:
            p.close()
    for r, c in enumerate(cases):
        g = op.Grid.from_case(c)
        ref, _ = rt.solve(g, rt.plane_wave(g), 1e-12, 3000)
        assert np.abs(got[r] - ref).max() <= 1e-8 * np.abs(ref).max(), r
