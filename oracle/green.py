"""Discretised dyadic Green's tensor T(m) and its circulant embedding.

Test infrastructure (see ``oracle/__init__``).

Sec. II-A, eq. (1): the scattered field of a polarisation current is
E^s = -j omega mu0 int G . J dv' with the dyadic Green's function
G = (I + grad grad / k^2) g and the scalar Green's function
g = exp(-j k R) / (4 pi R) (exp(+j omega t) convention).  Writing
J = j omega eps0 P turns this into E^s = k0^2 int G . P dv'.

Discretisation (collocated voxels, pulse basis, point matching): for a
non-zero voxel offset m the interaction is G sampled at the centre distance,
times the voxel volume; the self term is the integral of k0^2 G over a sphere
of the same volume as the voxel (principal value plus the -1/3 depolarisation),
which has the closed form (2/3)(1 + j k0 a) exp(-j k0 a) - 1.

Unique tensor components are stored in the order COMPONENTS =
(xx, xy, xz, yy, yz, zz).
"""
from __future__ import annotations

import numpy as np

COMPONENTS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def greens_tensor(Rx, Ry, Rz, k0: float, dV: float) -> np.ndarray:
    """k0^2 dV G(R) for non-zero separations R (eq. (1) with g after it).

    G(R) = g(R) [ (1 - j/u - 1/u^2) I + (3/u^2 + 3j/u - 1) Rhat Rhat ],
    u = k0 |R|, g = exp(-j u) / (4 pi |R|).  This is (I + grad grad/k0^2) g
    written out.  Returns an array of shape ``R.shape + (3, 3)``.
    """
    Rx = np.asarray(Rx, dtype=np.float64)
    Ry = np.asarray(Ry, dtype=np.float64)
    Rz = np.asarray(Rz, dtype=np.float64)
    R = np.sqrt(Rx * Rx + Ry * Ry + Rz * Rz)
    if np.any(R == 0):
        raise ValueError("greens_tensor: zero separation (use self_term)")
    u = k0 * R
    g = np.exp(-1j * u) / (4.0 * np.pi * R)
    a = 1.0 - 1j / u - 1.0 / (u * u)
    b = 3.0 / (u * u) + 3j / u - 1.0
    rh = (Rx / R, Ry / R, Rz / R)
    out = np.empty(R.shape + (3, 3), dtype=np.complex128)
    pref = k0 * k0 * dV * g
    for i in range(3):
        for j in range(3):
            out[..., i, j] = pref * ((1.0 if i == j else 0.0) * a + b * rh[i] * rh[j])
    return out


def self_term(dx: float, dy: float, dz: float, k0: float) -> complex:
    """Self interaction T(0) = t I of one voxel (scalar t returned).

    Integral of k0^2 G over the sphere of equal volume, radius
    a = (3 dV / 4 pi)^(1/3): t = (2 (1 + j k0 a) exp(-j k0 a) - 3) / 3.
    Static limit -1/3 (the depolarisation of a sphere).
    """
    dV = dx * dy * dz
    a = (3.0 * dV / (4.0 * np.pi)) ** (1.0 / 3.0)
    x = k0 * a
    return complex((2.0 * (1.0 + 1j * x) * np.exp(-1j * x) - 3.0) / 3.0)


def offset_tensor(mx, my, mz, dx, dy, dz, k0) -> np.ndarray:
    """T(m) for integer voxel offsets m (arrays), including m = 0."""
    mx = np.asarray(mx)
    my = np.asarray(my)
    mz = np.asarray(mz)
    shape = np.broadcast(mx, my, mz).shape
    mx = np.broadcast_to(mx, shape)
    my = np.broadcast_to(my, shape)
    mz = np.broadcast_to(mz, shape)
    out = np.zeros(shape + (3, 3), dtype=np.complex128)
    zero = (mx == 0) & (my == 0) & (mz == 0)
    nz_ = ~zero
    if np.any(nz_):
        out[nz_] = greens_tensor(mx[nz_] * dx, my[nz_] * dy, mz[nz_] * dz, k0, dx * dy * dz)
    if np.any(zero):
        out[zero] = self_term(dx, dy, dz, k0) * np.eye(3)
    return out


def circulant_offsets(n: int, L: int) -> np.ndarray:
    """Offset held by each slot of a length-L circulant embedding of an axis of n voxels.

    Slot s < n holds offset s, slot s > L - n holds offset s - L, the slots in
    between hold nothing (returned as a sentinel larger than any offset).
    Requires L >= 2n - 1 so positive and negative offsets do not overlap.
    """
    if L < 2 * n - 1:
        raise ValueError("circulant length too short")
    s = np.arange(L)
    off = np.full(L, 10 ** 9, dtype=np.int64)
    off[s < n] = s[s < n]
    neg = s > L - n
    off[neg] = s[neg] - L
    return off


def embedded_kernel(nx, ny, nz, dx, dy, dz, k0, L=None) -> np.ndarray:
    """The 6 unique components of T on the circulant-embedded grid.

    Default embedding length is L = 2n per axis with slot n left empty.
    Negative offsets are evaluated, not mirrored (T_xy is odd in m_x).
    Returns complex128 ``[6, Lz, Ly, Lx]``.
    """
    if L is None:
        L = (2 * nx, 2 * ny, 2 * nz)
    Lx, Ly, Lz = L
    ox = circulant_offsets(nx, Lx)
    oy = circulant_offsets(ny, Ly)
    oz = circulant_offsets(nz, Lz)
    big = 10 ** 9
    mz, my, mx = np.meshgrid(oz, oy, ox, indexing="ij")
    valid = (mx != big) & (my != big) & (mz != big)
    T = np.zeros((Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    T[valid] = offset_tensor(mx[valid], my[valid], mz[valid], dx, dy, dz, k0)
    out = np.empty((6, Lz, Ly, Lx), dtype=np.complex128)
    for c, (i, j) in enumerate(COMPONENTS):
        out[c] = T[..., i, j]
    return out
