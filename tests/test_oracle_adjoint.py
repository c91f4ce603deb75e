"""Pins of the adjoint oracle (Section 3.5): the Fourier coefficients of L*g,
hhat(xi) = (1/N) sum_y exp(-2 pi i Phi(y, xi)) g(y).

The adjoint is pinned against the forward oracle (itself pinned elsewhere)
through the defining identity <L fhat, g> = <fhat, L* g>, against closed
forms (Phi = x.xi makes L* the DFT of eq. (dft); an x-independent h makes it
a Fourier multiplier), against the conjugate transpose of the dense matrix,
and a planted missing conjugation must fail a pin.
"""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import direct as od
from oracle import reference as ref

FAMILIES = [(0, [0.13, -0.27]), (1, [0.05]), (2, [1.0]), (2, [1.4]), (3, [0.05, 0.5]), (4, [1.0]), (5, [1.0])]


@pytest.fixture(scope="module", autouse=True)
def _built():
    od.build(force=False)


@pytest.mark.parametrize("kind,p", FAMILIES)
def test_adjoint_identity_with_forward_oracle(kind, p):
    """<L fhat, g>_X = <fhat, L* g>_Omega on the whole grid (N = 32)."""
    N = 32
    rng = np.random.default_rng(31)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    g = fi.complex_gaussian(N, rng)
    u = od.direct(N, kind, p, fh, np.arange(N * N))
    h = od.direct_adjoint(N, kind, p, g, np.arange(N * N))
    lhs = np.vdot(g.ravel(), u)
    rhs = np.vdot(h, fh.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind,p", FAMILIES)
def test_adjoint_is_conjugate_transpose_of_dense_matrix(kind, p):
    N = 16
    rng = np.random.default_rng(32)
    g = fi.complex_gaussian(N, rng, B=2)
    K = ref.kernel_matrix(N, kind, p)
    h = od.direct_adjoint(N, kind, p, g, np.arange(N * N))
    for b in range(2):
        want = K.conj().T @ g[b].ravel()
        assert np.max(np.abs(h[b] - want)) < 1e-12 * np.max(np.abs(want))
    hn = ref.direct_adjoint(N, kind, p, g[0], np.arange(N * N))
    assert np.max(np.abs(hn - h[0])) < 1e-12 * np.max(np.abs(hn))


@pytest.mark.parametrize("N", [16, 32])
def test_adjoint_of_identity_phase_is_the_dft(N):
    """Phi = x.xi: L* g has the Fourier coefficients of eq. (dft) of g."""
    g = fi.complex_gaussian(N, np.random.default_rng(33))
    h = od.direct_adjoint(N, 0, [0.0, 0.0], g, np.arange(N * N)).reshape(N, N)
    assert np.max(np.abs(h - fi.fhat_from_f(g))) < 1e-12


@pytest.mark.parametrize("kind,p", [(1, [0.05]), (1, [-0.11]), (0, [0.0123, -0.371])])
def test_adjoint_multiplier_closed_form(kind, p):
    """x-independent h: hhat(xi) = exp(-2 pi i h(xi)) DFT(g)(xi), with numpy's FFT."""
    N = 32
    g = fi.complex_gaussian(N, np.random.default_rng(34))
    h = od.direct_adjoint(N, kind, p, g, np.arange(N * N)).reshape(N, N)
    k1, k2 = ref.grid_xi(N)
    mult = np.exp(-2j * np.pi * ref.h(kind, p, 0.0, 0.0, k1.astype(float), k2.astype(float))).reshape(N, N)
    want = mult * np.fft.fftshift(np.fft.fft2(g)) / N
    assert np.max(np.abs(h - want)) < 1e-11


def test_adjoint_of_a_multiplier_inverts_it():
    """For x-independent h the operator is unitary: L* L fhat = fhat."""
    N = 32
    fh = fi.fhat_from_f(fi.complex_gaussian(N, np.random.default_rng(35)))
    u = od.direct(N, 1, [0.07], fh, np.arange(N * N)).reshape(N, N)
    back = od.direct_adjoint(N, 1, [0.07], u, np.arange(N * N)).reshape(N, N)
    assert np.max(np.abs(back - fh)) < 1e-12


def test_adjoint_samples_match_full_grid():
    N = 32
    rng = np.random.default_rng(36)
    g = fi.complex_gaussian(N, rng, B=3)
    ks = np.sort(rng.choice(N * N, 50, replace=False))
    full = od.direct_adjoint(N, 2, [1.0], g, np.arange(N * N))
    part = od.direct_adjoint(N, 2, [1.0], g, ks)
    assert np.array_equal(part, full[:, ks])


def test_planted_missing_conjugation_is_caught(tmp_path):
    path = od.build(force=True, plant=6, out=str(tmp_path / "plant6.so"))
    N = 16
    g = fi.complex_gaussian(N, np.random.default_rng(37))
    h = od.direct_adjoint(N, 0, [0.0, 0.0], g, np.arange(N * N), lib_path=path).reshape(N, N)
    assert np.max(np.abs(h - fi.fhat_from_f(g))) > 1e-3
