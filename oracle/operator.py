"""The discretised VIE operator A of eqs. (2)-(4) and (6).

Test infrastructure (see ``oracle/__init__``).

For the unknown P = J / (j omega eps0) on the non-vacuum voxels S,

    (A P)_m = P_m / chi_m - sum_{n in S} T(m - n) P_n,   m in S,
    (A P)_m = 0,                                          m not in S,

with chi = eps_r - 1.  The first term is the constitutive relation eq. (2)
(E_tot = J / (j omega (eps - eps0)) = P / chi); the sum is the scattered
field of eq. (1); eq. (3) E_tot = E_inc + E^s then gives A P = E_inc, the
matrix equation (6).  Vacuum voxels carry no current (Sec. I: currents
between the dielectric and free space are not modelled) and are masked.

Three realisations of the same operator:

* ``dense_matrix``   assembled over S (tiny grids; LU reference);
* ``matvec_direct``  brute-force O(N^2) sum;
* ``matvec_fft``     the paper's FFT acceleration (Sec. I: the uniform grid
                     makes the matrix block-Toeplitz, so the product is a
                     zero-padded 3-D convolution done with FFTs).

Vectors are complex128 arrays ``[3, nz, ny, nx]`` (component-major, x fastest).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.fft

from .green import COMPONENTS, embedded_kernel, offset_tensor


@dataclasses.dataclass
class Grid:
    """A voxel grid with per-voxel relative permittivity."""

    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    wavelength: float
    eps: np.ndarray          # complex128 [nz, ny, nx]

    @property
    def k0(self) -> float:
        return 2.0 * np.pi / self.wavelength

    @property
    def dV(self) -> float:
        return self.dx * self.dy * self.dz

    @property
    def mask(self) -> np.ndarray:
        return self.eps != 1.0

    @property
    def chi(self) -> np.ndarray:
        return self.eps - 1.0

    @property
    def chi_inv(self) -> np.ndarray:
        """1 / chi on S, 0 on vacuum (where the equation is absent)."""
        out = np.zeros_like(self.eps)
        m = self.mask
        out[m] = 1.0 / (self.eps[m] - 1.0)
        return out

    @staticmethod
    def from_case(case) -> "Grid":
        return Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz,
                    case.wavelength, np.asarray(case.eps, dtype=np.complex128))


def _support(grid: Grid):
    k, j, i = np.nonzero(grid.mask)
    return i, j, k


def dense_matrix(grid: Grid):
    """Assemble A restricted to S.

    Returns ``(Z, idx)``: Z is complex128 of size 3|S| x 3|S| ordered
    component-major (all x unknowns, then y, then z), and idx the
    (i, j, k) voxel indices of S in that order.
    """
    i, j, k = _support(grid)
    n = i.size
    mx = i[:, None] - i[None, :]
    my = j[:, None] - j[None, :]
    mz = k[:, None] - k[None, :]
    T = offset_tensor(mx, my, mz, grid.dx, grid.dy, grid.dz, grid.k0)   # [n, n, 3, 3]
    chi_inv = grid.chi_inv[k, j, i]
    Z = np.empty((3 * n, 3 * n), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            Z[a * n:(a + 1) * n, b * n:(b + 1) * n] = -T[:, :, a, b]
    for a in range(3):
        Z[a * n + np.arange(n), a * n + np.arange(n)] += chi_inv
    return Z, (i, j, k)


def to_support(grid: Grid, x: np.ndarray, idx) -> np.ndarray:
    i, j, k = idx
    return np.concatenate([x[c][k, j, i] for c in range(3)])


def from_support(grid: Grid, v: np.ndarray, idx) -> np.ndarray:
    i, j, k = idx
    n = i.size
    out = np.zeros((3, grid.nz, grid.ny, grid.nx), dtype=np.complex128)
    for c in range(3):
        out[c][k, j, i] = v[c * n:(c + 1) * n]
    return out


def matvec_direct(grid: Grid, x: np.ndarray) -> np.ndarray:
    """(A x) by direct summation over all pairs of S (O(|S|^2))."""
    i, j, k = _support(grid)
    xs = np.stack([x[c][k, j, i] for c in range(3)], axis=-1)       # [n, 3]
    mx = i[:, None] - i[None, :]
    my = j[:, None] - j[None, :]
    mz = k[:, None] - k[None, :]
    T = offset_tensor(mx, my, mz, grid.dx, grid.dy, grid.dz, grid.k0)   # [n, n, 3, 3]
    field = np.einsum("mnab,nb->ma", T, xs)
    chi_inv = grid.chi_inv[k, j, i]
    ys = xs * chi_inv[:, None] - field
    out = np.zeros((3, grid.nz, grid.ny, grid.nx), dtype=np.complex128)
    for c in range(3):
        out[c][k, j, i] = ys[:, c]
    return out


def apply_at(grid: Grid, src: np.ndarray, xs: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """(A x) at the voxels ``dst`` [S, 3] (z, y, x) for an x that is zero
    except at the distinct voxels ``src`` [K, 3] (z, y, x), where it is
    ``xs`` [K, 3] (components x, y, z): the definition's direct sum over the
    K sources, for any grid size.  Returns [S, 3]."""
    src = np.asarray(src, dtype=np.int64).reshape(-1, 3)
    dst = np.asarray(dst, dtype=np.int64).reshape(-1, 3)
    xs = np.asarray(xs, dtype=np.complex128).reshape(-1, 3)
    eps_s = grid.eps[src[:, 0], src[:, 1], src[:, 2]]
    xs = np.where((eps_s != 1.0)[:, None], xs, 0.0)            # x lives on S only
    m = dst[:, None, :] - src[None, :, :]                       # [S, K, (z, y, x)]
    T = offset_tensor(m[..., 2], m[..., 1], m[..., 0], grid.dx, grid.dy, grid.dz, grid.k0)
    field = np.einsum("skab,kb->sa", T, xs)
    same = np.all(m == 0, axis=-1)                              # dst s is source k
    x_d = same.astype(np.complex128) @ xs
    eps_d = grid.eps[dst[:, 0], dst[:, 1], dst[:, 2]]
    on_s = eps_d != 1.0
    chi_inv = np.where(on_s, 1.0 / np.where(on_s, eps_d - 1.0, 1.0), 0.0)
    return np.where(on_s[:, None], x_d * chi_inv[:, None] - field, 0.0)


class FFTOperator:
    """A applied with the FFT convolution (Sec. I, Toeplitz + FFT).

    The 6 unique tensor components are embedded in a (2nz, 2ny, 2nx)
    circulant grid and transformed once.  A product zero-pads each masked
    component, transforms it, multiplies by the 3x3 symmetric spectrum,
    transforms back, crops to the original box and adds the local term.
    """

    def __init__(self, grid: Grid, pad: int = 0, product: str = "fp64"):
        # circulant length 2n (+ pad); any length >= 2n - 1 gives the same
        # product up to rounding (used to measure rounding sensitivity).
        # product="c64": the convolution (transforms and spectral multiply)
        # runs in complex64 and is widened again; the local term and every
        # vector operation stay FP64 (the mixed-precision mode).
        if product not in ("fp64", "c64"):
            raise ValueError(product)
        self.grid = grid
        self.product = product
        self.L = (2 * grid.nx + pad, 2 * grid.ny + pad, 2 * grid.nz + pad)
        kern = embedded_kernel(grid.nx, grid.ny, grid.nz, grid.dx, grid.dy, grid.dz, grid.k0, self.L)
        self.spec = scipy.fft.fftn(kern, axes=(1, 2, 3))
        if product == "c64":
            self.spec = self.spec.astype(np.complex64)
        self.mask = grid.mask
        self.chi_inv = grid.chi_inv

    def convolve(self, x: np.ndarray) -> np.ndarray:
        """sum_n T(m - n) x_n for every voxel m of the box (no mask on output)."""
        g = self.grid
        Lx, Ly, Lz = self.L
        dt = np.complex64 if self.product == "c64" else np.complex128
        xp = np.zeros((3, Lz, Ly, Lx), dtype=dt)
        xp[:, :g.nz, :g.ny, :g.nx] = x * self.mask
        X = scipy.fft.fftn(xp, axes=(1, 2, 3))
        Y = np.zeros_like(X)
        for c, (a, b) in enumerate(COMPONENTS):
            Y[a] += self.spec[c] * X[b]
            if a != b:
                Y[b] += self.spec[c] * X[a]
        y = scipy.fft.ifftn(Y, axes=(1, 2, 3))
        return y[:, :g.nz, :g.ny, :g.nx].astype(np.complex128)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        xm = x * self.mask
        return (xm * self.chi_inv - self.convolve(xm)) * self.mask


def matvec_fft(grid: Grid, x: np.ndarray) -> np.ndarray:
    return FFTOperator(grid)(x)
