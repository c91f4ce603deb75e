"""Pins of the deterministic preprocessing oracle (Section 3.1): the polar
Taylor coefficients of the residual phase, the compression of products of
separated expansions, and the separated approximation they build.

The coefficients are pinned by the closed form of the isotropic families
(phi_ell = a (1 - cos t), whose Taylor series is known term by term) and, for
the anisotropic ones, by a polynomial least-squares fit of phi_ell sampled on
the real angle (a different route to the same coefficients).  The
separation is pinned by the full SVD: its error falls with the Taylor
degree to the order of eps, its rank stays within two of the eps-rank, and
an x-independent phase gives rank one.
"""
import math

import numpy as np
import pytest

from oracle import reference as ref


@pytest.mark.parametrize("kind,p", [(3, [0.05, 0.5]), (5, [1.0]), (1, [0.07])])
def test_isotropic_coefficients_closed_form(kind, p):
    rng = np.random.default_rng(61)
    x1, x2 = rng.random(40), rng.random(40)
    theta_l = 0.7
    c = ref.taylor_coefficients(kind, p, x1, x2, theta_l, 8)
    a, _ = ref._coeffs(kind, np.asarray(p, float), x1, x2)
    a = np.broadcast_to(a, x1.shape)
    # 1 - cos t = t^2/2 - t^4/24 + t^6/720 - t^8/40320
    want = np.zeros((x1.size, 9))
    for k, v in ((2, 1 / 2), (4, -1 / 24), (6, 1 / 720), (8, -1 / 40320)):
        want[:, k] = a * v
    # the Cauchy integral on a circle of radius 1/4 scales rounding by 4^k
    tol = 1e-14 * 4.0 ** np.arange(9)
    assert np.all(np.abs(c - want) < tol[None, :])


@pytest.mark.parametrize("kind,p", [(2, [1.0]), (4, [1.0])])
def test_anisotropic_coefficients_against_polynomial_fit(kind, p):
    rng = np.random.default_rng(62)
    x1, x2 = rng.random(10), rng.random(10)
    theta_l = 1.1
    c = ref.taylor_coefficients(kind, p, x1, x2, theta_l, 5)
    t = np.linspace(-0.04, 0.04, 401)
    for i in range(x1.size):
        phi = ref.angular_residual(kind, p, x1[i], x2[i], theta_l + t, theta_l).real
        fit = np.polynomial.polynomial.polyfit(t, phi, 9)
        assert abs(c[i, 0]) < 1e-12 and abs(c[i, 1]) < 1e-10      # Phi_ell and its angular slope vanish at theta_l
        np.testing.assert_allclose(c[i, 2:4], fit[2:4], rtol=1e-5, atol=1e-9)


def test_compression_keeps_an_exact_low_rank_product():
    rng = np.random.default_rng(63)
    U = rng.standard_normal((300, 4)) + 1j * rng.standard_normal((300, 4))
    V = rng.standard_normal((4, 90)) + 1j * rng.standard_normal((4, 90))
    X = np.hstack([U, U @ rng.standard_normal((4, 6))])          # 10 columns, rank 4
    Y = np.vstack([V, np.zeros((6, 90))])
    Xc, Yc = ref._compress(X, Y, 1e-10)
    assert Xc.shape[1] == 4
    np.testing.assert_allclose(Xc @ Yc, X @ Y, atol=1e-10 * np.abs(X @ Y).max())


def _wedge(N, L, ell):
    ids, th = ref.equiangular_partition(N, L)
    k1, k2 = ref.grid_xi(N)
    sel = ids.ravel() == ell
    return th[ell], k1[sel], k2[sel]


@pytest.mark.parametrize("kind,p,eps", [(2, [1.0], 1e-4), (2, [1.0], 1e-6), (3, [0.05, 0.5], 1e-6), (5, [1.0], 1e-6)])
def test_taylor_separation_converges_and_matches_svd_rank(kind, p, eps):
    N, L = 32, 16
    for ell in (0, 5):
        th, k1, k2 = _wedge(N, L, ell)
        A = ref.residual_matrix(N, kind, p, th, np.arange(N * N), k1, k2)
        errs = []
        for pdeg in (1, 2, 3, 4, 5):
            r = ref.taylor_separation(N, kind, p, th, k1, k2, eps, pdeg)
            errs.append(np.linalg.norm(A - r["X"] @ r["Y"]) / np.linalg.norm(A))
        assert errs[-1] <= 3 * eps, errs
        assert errs[-1] <= errs[0]
        assert abs(r["q"] - ref.eps_rank(A, eps)) <= 2


def test_x_independent_phase_gives_rank_one():
    N, L = 32, 8
    th, k1, k2 = _wedge(N, L, 2)
    r = ref.taylor_separation(N, 1, [0.05], th, k1, k2, 1e-8, 4)
    A = ref.residual_matrix(N, 1, [0.05], th, np.arange(N * N), k1, k2)
    assert r["q"] == 1
    assert np.linalg.norm(A - r["X"] @ r["Y"]) / np.linalg.norm(A) < 1e-8
