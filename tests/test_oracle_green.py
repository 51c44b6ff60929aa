"""Pins of the oracle's Green tensor T(m) (eq. (1) and the scalar Green's
function after it) against facts fixed by the mathematics, not by retyping
its formula: a finite-difference evaluation of (I + grad grad / k^2) g, the
trace identity, symmetries, the static limit and a quadrature of the
self-cell integral."""
import numpy as np
import pytest
import scipy.fft
import scipy.integrate

from oracle import green


def _g(R, k):
    return np.exp(-1j * k * R) / (4 * np.pi * R)


def _fd_dyadic(r, k, h):
    """k^2 (I g + grad grad g / k^2) at point r, 4th-order central differences."""
    def gfun(p):
        return _g(np.linalg.norm(p), k)

    D = np.zeros((3, 3), dtype=complex)
    e = np.eye(3)
    for i in range(3):
        for j in range(3):
            if i == j:
                f = lambda t: gfun(r + t * e[i])
                D[i, i] = (-f(2 * h) + 16 * f(h) - 30 * f(0) + 16 * f(-h) - f(-2 * h)) / (12 * h * h)
            else:
                acc = 0
                for si, sj, w in [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]:
                    acc += w * gfun(r + si * h * e[i] + sj * h * e[j])
                D[i, j] = acc / (4 * h * h)
    return k * k * (np.eye(3) * gfun(r) + D / (k * k))


@pytest.mark.parametrize("r,k", [((0.3, -0.2, 0.45), 2 * np.pi), ((1.1, 0.7, -0.4), 5.0),
                                 ((0.05, 0.02, -0.03), 2 * np.pi / 0.9)])
def test_dyadic_matches_finite_differences(r, k):
    r = np.array(r)
    got = green.greens_tensor(r[0], r[1], r[2], k, 1.0)
    want = _fd_dyadic(r, k, 3e-4 * np.linalg.norm(r))  # O(h^2) stencil: ~3e-7
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def test_trace_identity():
    rng = np.random.default_rng(0)
    R = rng.uniform(-2, 2, (50, 3))
    k, dV = 3.7, 0.02
    T = green.greens_tensor(R[:, 0], R[:, 1], R[:, 2], k, dV)
    Rn = np.linalg.norm(R, axis=1)
    assert np.allclose(np.trace(T, axis1=1, axis2=2), 2 * k * k * dV * _g(Rn, k), rtol=1e-13, atol=0)


def test_symmetries_of_offsets():
    k0 = 2 * np.pi
    d = (0.05, 0.06, 0.045)
    m = np.array([(a, b, c) for a in range(-3, 4) for b in range(-3, 4) for c in range(-3, 4)])
    T = green.offset_tensor(m[:, 0], m[:, 1], m[:, 2], *d, k0)
    Tm = green.offset_tensor(-m[:, 0], -m[:, 1], -m[:, 2], *d, k0)
    assert np.allclose(T, np.swapaxes(T, 1, 2), rtol=0, atol=1e-15)
    assert np.allclose(T, Tm, rtol=0, atol=1e-15)
    Tx = green.offset_tensor(-m[:, 0], m[:, 1], m[:, 2], *d, k0)
    Ty = green.offset_tensor(m[:, 0], -m[:, 1], m[:, 2], *d, k0)
    Tz = green.offset_tensor(m[:, 0], m[:, 1], -m[:, 2], *d, k0)
    # parity: component ij is odd in axis a iff exactly one of i, j equals a
    for i in range(3):
        for j in range(3):
            for a, Ta in enumerate((Tx, Ty, Tz)):
                sgn = -1 if ((i == a) != (j == a)) else 1
                assert np.allclose(Ta[:, i, j], sgn * T[:, i, j], rtol=0, atol=1e-15)


def test_static_limit():
    k0 = 1e-5
    dV = 0.7
    R = np.array([0.3, -0.5, 0.2])
    T = green.greens_tensor(R[0], R[1], R[2], k0, dV)
    Rn = np.linalg.norm(R)
    rh = R / Rn
    static = dV * (3 * np.outer(rh, rh) - np.eye(3)) / (4 * np.pi * Rn ** 3)
    assert np.allclose(T, static, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("d,k0", [((1.0, 1.0, 1.0), 0.3), ((0.05, 0.05, 0.05), 2 * np.pi),
                                  ((0.03, 0.04, 0.025), 2 * np.pi), ((1.0, 1.0, 1.0), 1.5)])
def test_self_term_equals_sphere_integral(d, k0):
    """PV integral of k0^2 G over the equal-volume sphere, by quadrature.

    The angular mean of G(R) is (1/3) tr G = (2/3) g(R) I, and the static
    dyadic averages to zero, so the integral is
    -1/3 + (2/3) k0^2 int_0^a R exp(-j k0 R) dR   (the -1/3 is the delta term
    of grad grad (1/R)).
    """
    dV = d[0] * d[1] * d[2]
    a = (3 * dV / (4 * np.pi)) ** (1 / 3)
    re = scipy.integrate.quad(lambda R: R * np.cos(k0 * R), 0, a, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    im = scipy.integrate.quad(lambda R: -R * np.sin(k0 * R), 0, a, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    want = -1 / 3 + (2 / 3) * k0 * k0 * (re + 1j * im)
    assert abs(green.self_term(*d, k0) - want) <= 1e-12


def test_self_term_series():
    for x in [1e-3, 1e-2, 3e-2]:
        # k0 a = x with unit cube: a = (3/(4 pi))^(1/3)
        a = (3 / (4 * np.pi)) ** (1 / 3)
        t = green.self_term(1, 1, 1, x / a)
        series = -1 / 3 + x * x / 3 - 2j / 9 * x ** 3
        assert abs(t - series) <= 2 * x ** 4


def test_self_term_static_depolarisation():
    assert abs(green.self_term(1, 1, 1, 1e-9) + 1 / 3) < 1e-15


def test_circulant_slots():
    off = green.circulant_offsets(5, 10)
    assert list(off[:5]) == [0, 1, 2, 3, 4]
    assert off[5] == 10 ** 9
    assert list(off[6:]) == [-4, -3, -2, -1]
    odd = green.circulant_offsets(4, 7)
    assert list(odd) == [0, 1, 2, 3, -3, -2, -1]
    with pytest.raises(ValueError):
        green.circulant_offsets(5, 8)


def test_embedded_kernel_spectrum_parity():
    """Even/odd components give spectra with S(L - q) = +/- S(q) per axis."""
    n = (4, 3, 5)
    L = (8, 6, 10)
    k = green.embedded_kernel(*n, 0.05, 0.05, 0.05, 2 * np.pi, L)
    S = scipy.fft.fftn(k, axes=(1, 2, 3))
    for c, (i, j) in enumerate(green.COMPONENTS):
        for ax, arr_axis in ((0, 3), (1, 2), (2, 1)):
            sgn = -1 if ((i == ax) != (j == ax)) else 1
            flipped = np.roll(np.flip(S[c], axis=arr_axis - 1), 1, axis=arr_axis - 1)
            assert np.allclose(flipped, sgn * S[c], rtol=1e-12, atol=1e-12 * np.abs(S[c]).max())
