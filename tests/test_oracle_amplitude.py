"""Pins of the variable-amplitude oracle (Section 4, eq. (ellipses_amp), the
'+' amplitude a = (1/4pi)(J0(2 pi rho) + i Y0(2 pi rho)) exp(-2 pi i rho),
rho = h(x, xi), a(x, 0) = 0).

The C oracle takes J0 and Y0 from the C library and the NumPy one from
scipy.special.j0/y0.  Both are pinned against an independent construction of
the same function, the Hankel function H0^(1) = J0 + i Y0 of
scipy.special.hankel1, against its large-argument expansion (Abramowitz and
Stegun 9.2.3 with 9.2.5, 9.2.6) and small-argument form (9.1.13), and the
direct sum with the amplitude against the closed form of an x-independent
phase: a Fourier multiplier a(xi) exp(2 pi i h(xi)) applied with numpy's FFT.
"""
import math

import numpy as np
import pytest
from scipy import special

import fio_inputs as fi
from oracle import direct as od
from oracle import reference as ref


@pytest.fixture(scope="module", autouse=True)
def _built():
    od.build(force=False)


def _hankel_form(rho):
    z = 2 * np.pi * rho
    return special.hankel1(0, z) * np.exp(-1j * z) / (4 * np.pi)


@pytest.mark.parametrize("kind,p", [(1, [0.05]), (2, [1.0]), (3, [0.05, 0.5]), (4, [1.0]), (5, [1.0])])
def test_amplitude_equals_hankel_construction(kind, p):
    rng = np.random.default_rng(51)
    x1, x2 = rng.random(300), rng.random(300)
    k1, k2 = rng.integers(-400, 400, 300), rng.integers(-400, 400, 300)
    k1[0] = k2[0] = 0
    k1[1], k2[1] = 1, 0
    rho = ref.h(kind, p, x1, x2, k1, k2)
    want = _hankel_form(np.where(rho > 0, rho, 1.0))
    want[0] = 0
    ac = od.amp_values(kind, p, 1, x1, x2, k1, k2)
    an = ref.amplitude(kind, p, 1, x1, x2, k1, k2)
    scale = np.abs(want) + 1e-300
    assert np.max(np.abs(ac - want)[1:] / scale[1:]) < 1e-12
    assert np.max(np.abs(an - want)[1:] / scale[1:]) < 1e-12
    assert ac[0] == 0 and an[0] == 0


def test_amplitude_large_argument_expansion():
    """H0(z) exp(-iz) = sqrt(2/(pi z)) exp(-i pi/4) (P + iQ), P ~ 1 - 9/(128 z^2), Q ~ -1/(8z) + 75/(1024 z^3)."""
    rho = np.array([30.0, 100.0, 731.5])
    z = 2 * np.pi * rho
    P = 1 - 9 / (128 * z ** 2)
    Q = -1 / (8 * z) + 75 / (1024 * z ** 3)
    want = np.sqrt(2 / (np.pi * z)) * np.exp(-1j * np.pi / 4) * (P + 1j * Q) / (4 * np.pi)
    got = od.amp_values(1, [1.0], 1, 0 * rho, 0 * rho, rho, 0 * rho)   # wave phase, xi = (rho, 0): h = rho
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-8


def test_amplitude_small_argument_form():
    """J0(z) -> 1 and Y0(z) = (2/pi)(ln(z/2) + Euler's gamma) J0(z) + O(z^2) as z -> 0."""
    rho = 1e-7
    z = 2 * np.pi * rho
    want = (1 + 1j * (2 / np.pi) * (math.log(z / 2) + np.euler_gamma)) * np.exp(-1j * z) / (4 * np.pi)
    got = od.amp_values(1, [1e-7], 1, [0.0], [0.0], [1.0], [0.0])[0]
    assert abs(got - want) < 1e-10 * abs(want)


def test_amplitude_one_is_unity():
    a = od.amp_values(2, [1.0], 0, [0.1, 0.2], [0.3, 0.4], [0, 5], [0, -3])
    assert np.array_equal(a, np.ones(2, complex))


@pytest.mark.parametrize("ct", [0.05, 0.13])
def test_direct_sum_with_amplitude_multiplier_closed_form(ct):
    """Wave phase h = ct|xi| (x-independent) with the Bessel amplitude:
    u = IDFT(a(xi) exp(2 pi i h(xi)) DFT f), a from the Hankel construction."""
    N = 32
    f = fi.complex_gaussian(N, np.random.default_rng(52))
    fh = fi.fhat_from_f(f)
    u = od.direct(N, 1, [ct], fh, np.arange(N * N), amp=1).reshape(N, N)
    k1, k2 = ref.grid_xi(N)
    rho = ct * np.sqrt(k1 ** 2 + k2 ** 2.0)
    a = np.where(rho > 0, _hankel_form(np.where(rho > 0, rho, 1.0)), 0.0)
    mult = (a * np.exp(2j * np.pi * rho)).reshape(N, N)
    want = np.fft.ifft2(np.fft.ifftshift(np.fft.fftshift(np.fft.fft2(f)) * mult))
    assert np.max(np.abs(u - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("kind,p", [(5, [1.0]), (2, [1.0]), (4, [1.0])])
def test_c_and_numpy_amplitude_direct_sums_agree(kind, p):
    N = 24
    rng = np.random.default_rng(53)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    xs = fi.sample_points(N, 100, rng)
    uc = od.direct(N, kind, p, fh, xs, amp=1)
    un = ref.direct(N, kind, p, fh, xs, amp=1)
    assert ref.rel_l2(uc, un) < 1e-12


def test_adjoint_with_amplitude_identity():
    N = 24
    rng = np.random.default_rng(54)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    g = fi.complex_gaussian(N, rng)
    u = od.direct(N, 5, [1.0], fh, np.arange(N * N), amp=1)
    h = od.direct_adjoint(N, 5, [1.0], g, np.arange(N * N), amp=1)
    lhs, rhs = np.vdot(g.ravel(), u), np.vdot(h, fh.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
