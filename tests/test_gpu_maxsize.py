"""The product at the largest grid the library takes (256 cells per axis,
FFT 512^3), collocated and rooftop, against the oracle's direct sums at
sampled outputs for a sparse input: sources at the grid's corners and faces
(the largest offsets of the circulant embedding) and at random places;
outputs at the corners, the sources and random places.

Bars: max |GPU - oracle| over the samples / max |oracle| <= 1e-11 in FP64
(a 512^3 transform's rounding) and <= 1e-5 in mixed mode."""
import numpy as np
import pytest

import workloads as W
from oracle import operator as op, rooftop as rt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2501_13512_amd import vie as V  # noqa: E402

TOL = {V.VIE_FP64: 1e-11, V.VIE_MIXED: 1e-5}
N = 256


def _grid(c):
    return V.make_grid(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.wavelength)


def _corners(lo, hi):
    return np.array([[z, y, x] for z in (lo, hi) for y in (lo, hi) for x in (lo, hi)])


def test_collocated_product_at_the_largest_grid(vie_ctx):
    case = W.random_large(1)
    case.eps[tuple(_corners(0, N - 1).T)] = 3.0          # the corners are scatterer voxels
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(2)
    src = np.concatenate([_corners(0, N - 1), rng.integers(0, N, (56, 3))])
    src = np.unique(src, axis=0)
    xs = rng.standard_normal((len(src), 3)) + 1j * rng.standard_normal((len(src), 3))
    dst = np.concatenate([_corners(0, N - 1), src[:16], rng.integers(0, N, (40, 3))])
    want = op.apply_at(g, src, xs, dst)
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx)
    try:
        info = P.info()
        assert (info.lx, info.ly, info.lz) == (512, 512, 512)
        x = torch.zeros((3, N, N, N), dtype=torch.complex128, device="cuda")
        for c in range(3):
            x[c][tuple(torch.from_numpy(src.T))] = torch.from_numpy(xs[:, c].copy()).cuda()
        y = torch.empty_like(x)
        for prec in (V.VIE_FP64, V.VIE_MIXED):
            print(f"largest grid collocated prec {prec}", flush=True)
            V.vie_matvec(P.handle, prec, x, y)
            torch.cuda.synchronize()
            got = torch.stack([y[c][tuple(torch.from_numpy(dst.T))] for c in range(3)], dim=1).cpu().numpy()
            err = np.abs(got - want).max() / np.abs(want).max()
            print(f"  max rel err {err:.2e}", flush=True)
            assert err <= TOL[prec], (prec, err)
    finally:
        P.close()


def test_rooftop_product_at_the_largest_grid(vie_ctx):
    case = W.random_large(3, vacuum_shell=True)
    case.eps[tuple(_corners(1, N - 2).T)] = 3.0          # scatterer cells next to every corner of the shell
    g = op.Grid.from_case(case)
    rng = np.random.default_rng(4)
    # faces with unknowns: next to the shell's corners (lowest and highest
    # faces of every axis) and at random scatterer cells
    ext = []
    for z, y, x in _corners(1, N - 2):
        for c in range(3):
            ext.append((c, z, y, x))                        # face towards +c
            lo = np.array([z, y, x]) - rt._STEP[c]
            ext.append((c, *lo))                            # face towards -c (lower cell in the shell)
    cells = rng.integers(1, N - 1, (48, 3))
    rnd = np.concatenate([rng.integers(0, 3, (48, 1)), cells], axis=1)
    src = np.unique(np.concatenate([np.array(ext), rnd]), axis=0)
    src = src[rt.face_chi_at(g, src) != 0]
    vals = rng.standard_normal(len(src)) + 1j * rng.standard_normal(len(src))
    outs = np.concatenate([rng.integers(0, 3, (40, 1)), rng.integers(0, N, (40, 3))], axis=1)
    dst = np.concatenate([src[:24], outs, np.array(ext)])
    want = rt.apply_at(g, src, vals, dst)
    P = V.Problem(_grid(case), case.eps, ctx=vie_ctx, rooftop=True)
    try:
        info = P.info()
        assert (info.lx, info.ly, info.lz) == (512, 512, 512)
        x = torch.zeros((3, N, N, N), dtype=torch.complex128, device="cuda")
        x[tuple(torch.from_numpy(src.T))] = torch.from_numpy(vals).cuda()
        y = torch.empty_like(x)
        for prec in (V.VIE_FP64, V.VIE_MIXED):
            print(f"largest grid rooftop prec {prec}", flush=True)
            V.vie_matvec(P.handle, prec, x, y)
            torch.cuda.synchronize()
            got = y[tuple(torch.from_numpy(dst.T))].cpu().numpy()
            err = np.abs(got - want).max() / np.abs(want).max()
            print(f"  max rel err {err:.2e}", flush=True)
            assert err <= TOL[prec], (prec, err)
    finally:
        P.close()
