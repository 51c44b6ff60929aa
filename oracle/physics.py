"""Excitation, power balance, far field and the Mie series.

Test infrastructure (see ``oracle/__init__``).

* Plane wave: the structures of Sec. III are lit by an x-polarised wave
  travelling along z; E_inc = pol exp(-j k0 khat . r) (exp(+j omega t)),
  with the phase origin at the grid centre.
* Power terms, in units of k0 dV / (2 eta) (eta the free-space impedance):
  extinction  Im(P^H E_inc), absorption  sum Im(1/chi) |P|^2,
  scattering  -P^H Im(T) P.  For the discrete solution of A P = E_inc with
  complex-symmetric T they balance exactly (P_ext = P_abs + P_sca).
* The total field at every box voxel (incident plus scattered, eq. (3)).
* Far field of the voxel currents and the E-plane bistatic RCS used for the
  Mie comparison of Sec. III (Figs. 1-2).
* Mie series for a homogeneous sphere (the reference solution of Sec. III,
  ref. [30]), written from the textbook coefficients of Bohren & Huffman,
  "Absorption and Scattering of Light by Small Particles" (1983), ch. 4.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .operator import FFTOperator, Grid


def voxel_positions(grid: Grid):
    """Voxel-centre coordinates relative to the grid centre, each [nz, ny, nx]."""
    x = (np.arange(grid.nx) - (grid.nx - 1) / 2.0) * grid.dx
    y = (np.arange(grid.ny) - (grid.ny - 1) / 2.0) * grid.dy
    z = (np.arange(grid.nz) - (grid.nz - 1) / 2.0) * grid.dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def plane_wave(grid: Grid, kdir=(0.0, 0.0, 1.0), pol=(1.0, 0.0, 0.0)) -> np.ndarray:
    """E_inc at every voxel centre, complex128 [3, nz, ny, nx]."""
    X, Y, Z = voxel_positions(grid)
    phase = np.exp(-1j * grid.k0 * (kdir[0] * X + kdir[1] * Y + kdir[2] * Z))
    return np.stack([complex(p) * phase for p in pol])


def power_terms(grid: Grid, P: np.ndarray, e_inc: np.ndarray, op: FFTOperator = None):
    """(extinction, absorption, scattering) in units of k0 dV / (2 eta)."""
    if op is None:
        op = FFTOperator(grid)
    m = grid.mask
    Pm = P * m
    ext = float(np.imag(np.vdot(Pm.ravel(), (e_inc * m).ravel())))
    absn = float(np.sum(np.imag(grid.chi_inv[m]) * np.sum(np.abs(Pm[:, m]) ** 2, axis=0)))
    TP = op.convolve(Pm) * m
    # T complex symmetric => P^H Im(T) P = Im(P^H T P)
    sca = -float(np.imag(np.vdot(Pm.ravel(), TP.ravel())))
    return ext, absn, sca


def total_field_box(grid: Grid, P: np.ndarray, e_inc: np.ndarray) -> np.ndarray:
    """E_tot at every voxel of the box, scatterer or not: E_inc plus the
    scattered field sum_n T(m - n) P_n (eq. (3) with the discretised
    operator of eq. (1)).  On the scatterer this equals P / chi for the
    solution of A P = E_inc (eq. (2))."""
    return e_inc + FFTOperator(grid).convolve(P * grid.mask)


def far_field_vector(grid: Grid, P: np.ndarray, rhat: np.ndarray) -> np.ndarray:
    """F(rhat) = (I - rhat rhat) sum_n P_n dV exp(+j k0 rhat . r_n), rhat [..., 3]."""
    X, Y, Z = voxel_positions(grid)
    m = grid.mask
    pos = np.stack([X[m], Y[m], Z[m]], axis=-1)              # [n, 3]
    Pn = np.stack([P[c][m] for c in range(3)], axis=-1)      # [n, 3]
    rh = np.asarray(rhat, dtype=np.float64)
    flat = rh.reshape(-1, 3)
    out = np.empty(flat.shape, dtype=np.complex128)
    for s in range(0, flat.shape[0], 256):
        r = flat[s:s + 256]
        ph = np.exp(1j * grid.k0 * (r @ pos.T))             # [b, n]
        F = ph @ Pn * grid.dV                                # [b, 3]
        F = F - r * np.sum(r * F, axis=-1, keepdims=True)
        out[s:s + 256] = F
    return out.reshape(rh.shape)


def rcs_eplane(grid: Grid, P: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Bistatic RCS sigma(theta) in the E-plane (phi = 0, x-z plane).

    sigma = 4 pi r^2 |E^s|^2 / |E_inc|^2 with E^s = k0^2 G_far . sum P dV, i.e.
    sigma = k0^4 |F|^2 / (4 pi) for unit incident amplitude.
    """
    rh = np.stack([np.sin(theta), np.zeros_like(theta), np.cos(theta)], axis=-1)
    F = far_field_vector(grid, P, rh)
    return grid.k0 ** 4 * np.sum(np.abs(F) ** 2, axis=-1) / (4.0 * np.pi)


def scattered_power_far(grid: Grid, P: np.ndarray, n_theta: int = 48, n_phi: int = 96) -> float:
    """Scattering term from the far field, same units as ``power_terms``.

    (k0^3 / (16 pi^2 dV)) * integral over the sphere of |F|^2, by Gauss-Legendre
    in cos(theta) and the trapezoid rule in phi.
    """
    mu, w = np.polynomial.legendre.leggauss(n_theta)
    phi = np.arange(n_phi) * (2.0 * np.pi / n_phi)
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    st = np.sqrt(1.0 - MU * MU)
    rh = np.stack([st * np.cos(PHI), st * np.sin(PHI), MU], axis=-1)
    F = far_field_vector(grid, P, rh)
    I = np.sum(np.abs(F) ** 2, axis=-1)
    integral = float(np.sum(I * w[:, None]) * (2.0 * np.pi / n_phi))
    return grid.k0 ** 3 * integral / (16.0 * np.pi ** 2 * grid.dV)


def cross_sections(grid: Grid, P: np.ndarray, e_inc: np.ndarray):
    """(sigma_ext, sigma_abs, sigma_sca) for unit incident amplitude."""
    ext, absn, sca = power_terms(grid, P, e_inc)
    f = grid.k0 * grid.dV
    return ext * f, absn * f, sca * f


# --------------------------------------------------------------------------
# Mie series (Bohren & Huffman 1983, sec. 4.4 and 4.8), exp(-i omega t) form.
# --------------------------------------------------------------------------

def _riccati(n, z):
    """psi_n(z) = z j_n(z) and its derivative."""
    j = sp.spherical_jn(n, z)
    jd = sp.spherical_jn(n, z, derivative=True)
    return z * j, j + z * jd


def _riccati_h(n, x):
    """xi_n(x) = x h_n^(1)(x) and its derivative, real x."""
    h = sp.spherical_jn(n, x) + 1j * sp.spherical_yn(n, x)
    hd = sp.spherical_jn(n, x, derivative=True) + 1j * sp.spherical_yn(n, x, derivative=True)
    return x * h, h + x * hd


def mie_coefficients(m: complex, x: float, nmax: int = None):
    """Scattering coefficients a_n, b_n, n = 1..nmax, for relative index m and
    size parameter x (B&H eq. 4.53 with equal permeabilities)."""
    if nmax is None:
        nmax = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    n = np.arange(1, nmax + 1)
    mx = m * x
    psi_x, dpsi_x = _riccati(n, x)
    psi_mx, dpsi_mx = _riccati(n, mx)
    xi_x, dxi_x = _riccati_h(n, x)
    a = (m * psi_mx * dpsi_x - psi_x * dpsi_mx) / (m * psi_mx * dxi_x - xi_x * dpsi_mx)
    b = (psi_mx * dpsi_x - m * psi_x * dpsi_mx) / (psi_mx * dxi_x - m * xi_x * dpsi_mx)
    return a, b


def mie_efficiencies(m: complex, x: float):
    """(Q_ext, Q_sca) (B&H eqs. 4.61, 4.62)."""
    a, b = mie_coefficients(m, x)
    n = np.arange(1, a.size + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qsca)


def mie_amplitudes(m: complex, x: float, theta: np.ndarray):
    """S1(theta), S2(theta) (B&H eq. 4.74) with the angular functions pi_n,
    tau_n from their upward recurrences (B&H eq. 4.47)."""
    a, b = mie_coefficients(m, x)
    nmax = a.size
    mu = np.cos(theta)
    S1 = np.zeros(theta.shape, dtype=np.complex128)
    S2 = np.zeros(theta.shape, dtype=np.complex128)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    for n in range(1, nmax + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_cur)
        pi_next = ((2 * n + 1) * mu * pi_cur - (n + 1) * pi_prev) / n
        pi_prev, pi_cur = pi_cur, pi_next
    return S1, S2


def mie_rcs_eplane(eps_r: complex, radius: float, wavelength: float, theta: np.ndarray) -> np.ndarray:
    """E-plane bistatic RCS of a sphere: sigma = lambda^2 |S2|^2 / pi.

    ``eps_r`` is given in the paper's exp(+j omega t) convention (lossy:
    negative imaginary part) and conjugated for the exp(-i omega t) series.
    """
    m = np.sqrt(np.conj(complex(eps_r)))
    x = 2.0 * np.pi * radius / wavelength
    _, S2 = mie_amplitudes(m, x, theta)
    return wavelength ** 2 * np.abs(S2) ** 2 / np.pi
