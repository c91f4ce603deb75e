"""NumPy FP64 oracle for the wedge-localised FIO -- TEST INFRASTRUCTURE ONLY.

Every function here follows the paper's definitions and steps in plain
NumPy; nothing is blocked, fused or reordered beyond what the definition
states.  It shares no code with the HIP library (see oracle/__init__.py).

Conventions (Section 1.2): X = {(n1/N, n2/N)}, Omega = [-N/2, N/2)^2 with
N even; spatial arrays are indexed [n1, n2] (flat n1*N + n2); frequency
arrays are centred, [k1 + N/2, k2 + N/2].  Phases have the form
Phi(x, xi) = x.xi + h(x, xi) with h homogeneous of degree one in xi; the
family numbering matches oracle/direct.c.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
KINDS = {"linear": 0, "wave": 1, "c1c2": 2, "radial": 3, "paper_ellipse": 4, "paper_circle": 5}


# --------------------------------------------------------------------------
# Grids (Section 1.2)
# --------------------------------------------------------------------------
def grid_x(N):
    """Flat arrays (x1, x2) of X in row-major order (index n1*N + n2)."""
    n = np.arange(N) / N
    x1, x2 = np.meshgrid(n, n, indexing="ij")
    return x1.ravel(), x2.ravel()


def grid_xi(N):
    """Flat integer arrays (k1, k2) of Omega in the centred order."""
    k = np.arange(-N // 2, N // 2)
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    return k1.ravel(), k2.ravel()


def x_of_index(N, xidx):
    xidx = np.asarray(xidx, dtype=np.int64)
    return (xidx // N) / N, (xidx % N) / N


def dft_direct(f):
    """Eq. (dft) written out: fhat(xi) = (1/N) sum_x exp(-2 pi i x.xi) f(x), centred."""
    N = f.shape[0]
    x1, x2 = grid_x(N)
    k1, k2 = grid_xi(N)
    ph = np.outer(k1, x1) + np.outer(k2, x2)
    return (np.exp(-2j * np.pi * ph) @ f.ravel()).reshape(N, N) / N


# --------------------------------------------------------------------------
# Phase families: h(x, xi) and its xi-gradient
# --------------------------------------------------------------------------
def _coeffs(kind, p, x1, x2):
    """(a, b) of the ellipse-type families, h = p0 sqrt(a^2 xi1^2 + b^2 xi2^2),
    or (a, a) of the isotropic ones, h = a |xi| (a may carry a sign)."""
    if kind == 2:
        c1 = (2.0 + np.sin(TWO_PI * x1) * np.sin(TWO_PI * x2)) / 16.0
        c2 = (2.0 + np.cos(TWO_PI * x1) * np.cos(TWO_PI * x2)) / 16.0
        return c1, c2
    if kind == 4:
        r1 = (2.0 + np.sin(2 * TWO_PI * x1)) * (2.0 + np.sin(2 * TWO_PI * x2)) / 9.0
        r2 = (2.0 + np.cos(2 * TWO_PI * x1)) * (2.0 + np.cos(2 * TWO_PI * x2)) / 9.0
        return r1, r2
    if kind == 1:
        z = np.zeros_like(np.asarray(x1, dtype=float)) + p[0]
        return z, z
    if kind == 3:
        rho = p[0] * (1.0 + p[1] * np.sin(TWO_PI * x1))
        return rho, rho
    if kind == 5:
        r = p[0] * (3.0 + np.sin(2 * TWO_PI * x1)) * (3.0 + np.sin(2 * TWO_PI * x2)) / 16.0
        return r, r
    raise ValueError(kind)


def h(kind, p, x1, x2, k1, k2):
    """h(x, xi), so that Phi = x.xi + h; homogeneous of degree 1 in xi.

    linear: p0 xi1 + p1 xi2; ellipse families: p0 sqrt(a^2 xi1^2 + b^2 xi2^2)
    with (a, b) from `_coeffs`; isotropic families: a |xi| (a may be
    negative, e.g. the '-' wave phase).
    """
    p = np.asarray(p, dtype=float)
    if kind == 0:
        return p[0] * np.asarray(k1, float) + p[1] * np.asarray(k2, float)
    a, b = _coeffs(kind, p, x1, x2)
    k1 = np.asarray(k1, float)
    k2 = np.asarray(k2, float)
    if kind in (1, 3, 5):
        return a * np.sqrt(k1 * k1 + k2 * k2)
    return p[0] * np.sqrt(a * a * k1 * k1 + b * b * k2 * k2)


def grad_h(kind, p, x1, x2, e1, e2):
    """grad_xi h(x, xi) at xi = (e1, e2) (any nonzero vector; degree-0 homogeneous)."""
    p = np.asarray(p, dtype=float)
    e1 = np.asarray(e1, float)
    e2 = np.asarray(e2, float)
    if kind == 0:
        z = np.zeros(np.broadcast(np.asarray(x1), e1).shape)
        return z + p[0], z + p[1]
    a, b = _coeffs(kind, p, x1, x2)
    if kind in (1, 3, 5):
        r = np.sqrt(e1 * e1 + e2 * e2)
        return a * e1 / r, a * e2 / r
    q = np.sqrt(a * a * e1 * e1 + b * b * e2 * e2)
    return p[0] * a * a * e1 / q, p[0] * b * b * e2 / q


def amplitude(kind, p, amp, x1, x2, k1, k2):
    """a(x, xi): 1 (amp = 0), or the Bessel amplitude of Section 4 (amp = 1),
    a = (1/4 pi)(J0(2 pi rho) + i Y0(2 pi rho)) exp(-2 pi i rho) with rho =
    h(x, xi) >= 0, and a = 0 at xi = 0 (Y0 is singular there; the paper
    states no value).  J0 and Y0 from scipy.special."""
    from scipy import special
    k1 = np.asarray(k1, float)
    k2 = np.asarray(k2, float)
    if amp == 0:
        return np.ones(np.broadcast(np.asarray(x1), k1, k2).shape, dtype=complex)
    rho = h(kind, p, x1, x2, k1, k2)
    origin = (k1 == 0) & (k2 == 0)
    z = 2 * np.pi * np.where(origin, 1.0, rho)
    a = (special.j0(z) + 1j * special.y0(z)) * _expi(-rho) / (4 * np.pi)
    return np.where(origin, 0.0, a)


def phase(kind, p, x1, x2, k1, k2):
    """Phi(x, xi) = x.xi + h(x, xi) in FP64."""
    return np.asarray(x1) * k1 + np.asarray(x2) * k2 + h(kind, p, x1, x2, k1, k2)


def _expi(ph):
    """exp(2 pi i ph) after reduction by the nearest integer."""
    r = ph - np.rint(ph)
    return np.exp(2j * np.pi * r)


# --------------------------------------------------------------------------
# The operator itself (eq. dfio, Egorov form a = 1)
# --------------------------------------------------------------------------
def kernel_matrix(N, kind, p):
    """Dense N^2 x N^2 matrix K[x, xi] = exp(2 pi i Phi(x, xi)) / N (tiny N only)."""
    if N > 48:
        raise ValueError("dense matrix form is for N <= 48")
    x1, x2 = grid_x(N)
    k1, k2 = grid_xi(N)
    X1, K1 = np.meshgrid(x1, k1, indexing="ij")
    X2, K2 = np.meshgrid(x2, k2, indexing="ij")
    return _expi(phase(kind, p, X1, X2, K1, K2)) / N


def apply_dense(N, kind, p, fhat):
    """u = K fhat over the whole grid via the dense matrix (tiny N)."""
    return (kernel_matrix(N, kind, p) @ np.asarray(fhat).reshape(N * N)).reshape(N, N)


def direct(N, kind, p, fhat, xidx, member=None, only=0, chunk=64, amp=0):
    """(Lf)(x) at flat indices `xidx` by FP64 direct sum over Omega (or one wedge).

    Independent of the C oracle: vectorised NumPy with a per-chunk matrix.
    amp = 1 multiplies the kernel by the Bessel amplitude (`amplitude`).
    """
    fh = np.asarray(fhat, dtype=np.complex128).reshape(N * N)
    k1, k2 = grid_xi(N)
    if member is not None:
        sel = np.asarray(member).reshape(N * N) == only
        k1, k2, fh = k1[sel], k2[sel], fh[sel]
    x1, x2 = x_of_index(N, xidx)
    out = np.empty(x1.size, dtype=np.complex128)
    for s in range(0, x1.size, chunk):
        a1 = x1[s:s + chunk, None]
        a2 = x2[s:s + chunk, None]
        K = _expi(phase(kind, p, a1, a2, k1[None, :], k2[None, :]))
        if amp:
            K = K * amplitude(kind, p, amp, a1, a2, k1[None, :], k2[None, :])
        out[s:s + chunk] = K @ fh / N
    return out


def direct_adjoint(N, kind, p, g, xiidx, chunk=64):
    """Fourier coefficients of L*g at flat centred indices `xiidx` (Section 3.5):
    hhat(xi) = (1/N) sum_y exp(-2 pi i Phi(y, xi)) g(y), vectorised NumPy."""
    gv = np.asarray(g, dtype=np.complex128).reshape(N * N)
    x1, x2 = grid_x(N)
    xiidx = np.asarray(xiidx, dtype=np.int64)
    k1 = xiidx // N - N // 2
    k2 = xiidx % N - N // 2
    out = np.empty(xiidx.size, dtype=np.complex128)
    for s in range(0, xiidx.size, chunk):
        a1 = k1[s:s + chunk, None].astype(float)
        a2 = k2[s:s + chunk, None].astype(float)
        out[s:s + chunk] = np.conj(_expi(phase(kind, p, x1[None, :], x2[None, :], a1, a2))) @ gv / N
    return out


def multiplier_solution(N, hfun, f):
    """Closed form for Phi = x.xi + h(xi) (x-independent h): u = IDFT(e^{2 pi i h(xi)} DFT f).

    Uses the centred representative xi in [-N/2, N/2)^2 (h is not N-periodic),
    with numpy's FFT as the library routine for both transforms.
    """
    F = np.fft.fftshift(np.fft.fft2(f))
    k1, k2 = grid_xi(N)
    mult = np.exp(2j * np.pi * hfun(k1.astype(float), k2.astype(float))).reshape(N, N)
    return np.fft.ifft2(np.fft.ifftshift(F * mult))


# --------------------------------------------------------------------------
# Wedge partitions (Section 1.3)
# --------------------------------------------------------------------------
def equiangular_partition(N, L):
    """Wedge id per centred frequency and centre angles theta_ell = 2 pi ell / L.

    W_ell = {(2 ell - 1) pi/L <= arg xi < (2 ell + 1) pi/L} with arg in
    [0, 2 pi); xi = 0 is assigned to wedge 0.
    """
    k1, k2 = grid_xi(N)
    arg = np.mod(np.arctan2(k2.astype(float), k1.astype(float)), TWO_PI)
    width = TWO_PI / L
    ids = np.floor((arg + math.pi / L) / width).astype(np.int64) % L
    ids[(k1 == 0) & (k2 == 0)] = 0
    thetas = TWO_PI * np.arange(L) / L
    return ids.reshape(N, N).astype(np.int32), thetas


def corona_partition(N):
    """Dyadic coronae split into angular wedges (the multiscale variant).

    Corona 0 is |xi| < 8 (with xi = 0); corona j >= 1 is 2^(j+2) <= |xi| <
    2^(j+3).  Corona j is cut into n_j = 8 * 2^ceil(j/2) equiangular wedges
    centred at 2 pi k / n_j, with the same half-open rule as
    `equiangular_partition`.  Wedge ids run corona by corona.  Returns
    (ids (N, N) int32, thetas) with one theta per wedge id.
    """
    k1, k2 = grid_xi(N)
    rad = np.sqrt(k1.astype(float) ** 2 + k2.astype(float) ** 2)
    rmax = rad.max()
    arg = np.mod(np.arctan2(k2.astype(float), k1.astype(float)), TWO_PI)
    ids = np.empty(k1.size, dtype=np.int64)
    thetas = []
    j = 0
    base = 0
    while True:
        lo = 0.0 if j == 0 else 2.0 ** (j + 2)
        hi = 2.0 ** (j + 3)
        if lo > rmax:
            break
        nj = 8 * 2 ** ((j + 1) // 2)
        sel = (rad >= lo) & (rad < hi)
        width = TWO_PI / nj
        kk = np.floor((arg[sel] + math.pi / nj) / width).astype(np.int64) % nj
        ids[sel] = base + kk
        thetas.extend(TWO_PI * np.arange(nj) / nj)
        base += nj
        j += 1
    ids[(k1 == 0) & (k2 == 0)] = 0
    return ids.reshape(N, N).astype(np.int32), np.asarray(thetas)


# --------------------------------------------------------------------------
# Linearisation and residual phase (Section 1.3)
# --------------------------------------------------------------------------
def warp(kind, p, x1, x2, theta):
    """Warped point y = grad_xi Phi(x, xi_hat) = x + grad_xi h(x, xi_hat)."""
    g1, g2 = grad_h(kind, p, x1, x2, math.cos(theta), math.sin(theta))
    return np.asarray(x1) + g1, np.asarray(x2) + g2


def residual_phase(kind, p, x1, x2, k1, k2, theta):
    """Phi_ell(x, xi) = Phi(x, xi) - grad_xi Phi(x, xi_hat_ell).xi = h - grad h(xi_hat).xi."""
    g1, g2 = grad_h(kind, p, x1, x2, math.cos(theta), math.sin(theta))
    return h(kind, p, x1, x2, k1, k2) - (g1 * k1 + g2 * k2)


def residual_matrix(N, kind, p, theta, xidx, k1, k2):
    """A[x, xi] = exp(2 pi i Phi_ell(x, xi)) for x in xidx, xi in (k1, k2) (eq. probform)."""
    x1, x2 = x_of_index(N, xidx)
    ph = residual_phase(kind, p, x1[:, None], x2[:, None], np.asarray(k1, float)[None, :],
                        np.asarray(k2, float)[None, :], theta)
    return _expi(ph)


# --------------------------------------------------------------------------
# Randomized separation (Section 3.2)
# --------------------------------------------------------------------------
def randomized_separation(N, kind, p, theta, k1, k2, eps, rng, r0=48, accept=1.0 / 3.0):
    """Low-rank A ~ U T of A = exp(2 pi i Phi_ell) on X x W_ell, by the paper's steps.

    1. choose r columns C of A uniformly at random (without replacement);
    2. SVD of A_[C], keeping singular values above eps * s_1 (relative
       reading of the threshold);
    3. if q > r * accept, double r and restart;
    4. choose r rows R uniformly at random; T = pinv(U_[R]) A_[R].
    The paper leaves the starting r open ("begin with a small r"); 48 is
    used here because uniform samples of 12-24 columns leave holes in the
    wedge at eps <= 1e-4 (errors of 5-20 eps were observed).
    Returns dict(U (N^2 x q), T (q x n), q, r, C, R, s (singular values)).
    """
    n = len(k1)
    m = N * N
    allx = np.arange(m)
    k1 = np.asarray(k1)
    k2 = np.asarray(k2)
    r = r0
    while True:
        rc = min(r, n)
        C = np.sort(rng.choice(n, size=rc, replace=False))
        AC = residual_matrix(N, kind, p, theta, allx, k1[C], k2[C])
        Uf, s, _ = np.linalg.svd(AC, full_matrices=False)
        q = int(np.count_nonzero(s > eps * s[0]))
        if q <= r * accept or rc >= n:
            break
        r *= 2
    U = Uf[:, :q]
    R = np.sort(rng.choice(m, size=min(r, m), replace=False))
    AR = residual_matrix(N, kind, p, theta, R, k1, k2)
    T = np.linalg.pinv(U[R], rcond=1e-12) @ AR
    return dict(U=U, T=T, q=q, r=r, C=C, R=R, s=s)


# --------------------------------------------------------------------------
# Deterministic preprocessing (Section 3.1): Taylor expansions and
# QR + SVD compression of products of separated expansions
# --------------------------------------------------------------------------
def angular_residual(kind, p, x1, x2, theta, theta_l):
    """phi_ell(x, theta) = Phi_ell(x, xi) / |xi| for xi = |xi| (cos theta, sin theta):
    h(x, e(theta)) - grad_xi h(x, e(theta_l)) . e(theta), valid for complex theta."""
    e1, e2 = np.cos(theta), np.sin(theta)
    g1, g2 = grad_h(kind, p, x1, x2, math.cos(theta_l), math.sin(theta_l))
    a, b = _coeffs(kind, np.asarray(p, float), x1, x2) if kind != 0 else (None, None)
    if kind == 0:
        hv = p[0] * e1 + p[1] * e2
    elif kind in (1, 3, 5):
        hv = a * np.sqrt(e1 * e1 + e2 * e2 + 0j)
    else:
        hv = p[0] * np.sqrt(a * a * e1 * e1 + b * b * e2 * e2 + 0j)
    return hv - (g1 * e1 + g2 * e2)


def taylor_coefficients(kind, p, x1, x2, theta_l, K, radius=0.25, M=64):
    """c_k(x), k = 0..K, of phi_ell(x, theta_l + t) = sum_k c_k t^k: the Cauchy
    integral of phi_ell over a circle of the given radius around theta_l,
    evaluated by the trapezoidal rule at M points (exact for the analytic
    phi to about (radius / R)^M, R the distance to its nearest singularity).
    Returns (len(x), K + 1)."""
    z = radius * np.exp(2j * np.pi * np.arange(M) / M)
    vals = angular_residual(kind, p, np.asarray(x1)[:, None], np.asarray(x2)[:, None], theta_l + z[None, :], theta_l)
    coef = np.fft.fft(vals, axis=1) / M
    k = np.arange(K + 1)
    return (coef[:, :K + 1] / radius ** k[None, :]).real


def _compress(X, Y, eps):
    """X Y ~ X~ Y~ with fewer columns: QR of X and of Y^T, SVD of R_X R_Y^T,
    singular values below eps * s_1 dropped (Section 3.1's compression)."""
    QX, RX = np.linalg.qr(X)
    QY, RY = np.linalg.qr(Y.T)
    U, S, Vh = np.linalg.svd(RX @ RY.T)
    q = max(1, int(np.count_nonzero(S > eps * S[0])))
    return QX @ (U[:, :q] * S[:q]), Vh[:q] @ QY.T


def taylor_separation(N, kind, p, theta_l, k1, k2, eps, pdeg=3, xidx=None):
    """Deterministic separated approximation of A = exp(2 pi i Phi_ell) on
    X x W_ell (Section 3.1), in the paper's steps:
      1. Phi_ell(x, xi) ~ |xi| sum_{k=1}^{2p+1} c_k(x) (theta - theta_ell)^k;
      2. for each k, exp(2 pi i c_k(x) |xi| (theta - theta_ell)^k) ~
         sum_{m < d_k} beta^x_km(x) beta^xi_km(xi) by truncating the Taylor
         series of the exponential (d_k: the first m with z^m / m! below
         eps / 10, z the largest |2 pi c_k(x) |xi| (theta - theta_ell)^k|);
      3. the expansions are multiplied two by two and each product is
         compressed (QR and SVD, threshold eps relative to the largest
         singular value).
    Returns dict(X (n_x x q), Y (q x n_xi), q, ranks per product)."""
    if xidx is None:
        xidx = np.arange(N * N)
    x1, x2 = x_of_index(N, xidx)
    k1 = np.asarray(k1, float)
    k2 = np.asarray(k2, float)
    rad = np.sqrt(k1 * k1 + k2 * k2)
    th = np.arctan2(k2, k1)
    dth = np.angle(np.exp(1j * (th - theta_l)))
    K = 2 * pdeg + 1
    c = taylor_coefficients(kind, p, x1, x2, theta_l, K)
    X = np.ones((x1.size, 1), complex)
    Y = np.ones((1, k1.size), complex)
    ranks = []
    for k in range(1, K + 1):
        tk = rad * dth ** k                      # |xi| (theta - theta_ell)^k
        scale = max(np.max(np.abs(tk)), 1e-300)
        zx = 2j * np.pi * c[:, k] * scale        # so that beta^xi = (tk / scale)^m is at most 1
        zmax = np.max(np.abs(zx))
        d = 1
        term = 1.0
        while term > eps / 10 and d < 200:
            term *= zmax / d
            d += 1
        m = np.arange(d)
        fact = np.array([math.factorial(int(v)) for v in m], float)
        Bx = zx[:, None] ** m[None, :] / fact[None, :]
        Bxi = (tk / scale)[None, :] ** m[:, None]
        # product with the running expansion, then compression
        Xp = (X[:, :, None] * Bx[:, None, :]).reshape(x1.size, -1)
        Yp = (Y[:, None, :] * Bxi[None, :, :]).reshape(-1, k1.size)
        X, Y = _compress(Xp, Yp, eps)
        ranks.append(X.shape[1])
    return dict(X=X, Y=Y, q=X.shape[1], ranks=ranks)


def separation_error(N, kind, p, theta, k1, k2, U, T, rng, s=200):
    """Estimator of Section 4: ||A_GD - U_G T_D||_F / ||A_GD||_F on random s x s."""
    m = N * N
    n = len(k1)
    G = np.sort(rng.choice(m, size=min(s, m), replace=False))
    D = np.sort(rng.choice(n, size=min(s, n), replace=False))
    A = residual_matrix(N, kind, p, theta, G, np.asarray(k1)[D], np.asarray(k2)[D])
    E = A - U[G] @ T[:, D]
    return float(np.linalg.norm(E) / np.linalg.norm(A))


def eps_rank(A, eps):
    """Number of singular values of A above eps * s_1 (full SVD)."""
    s = np.linalg.svd(A, compute_uv=False)
    return int(np.count_nonzero(s > eps * s[0]))


def lemma1_rank_bound(A, eps):
    """Lemma 1: eps-rank bound of exp(i x y) on [-A, A] x [-1, 1]."""
    if A <= 1.0 / (2.0 * math.e):
        return 1.0 + math.log(2.0 / eps) / math.log(1.0 / (math.e * A))
    return 1.0 + max(2.0 * math.e * A, math.log2(2.0 / eps))


# --------------------------------------------------------------------------
# Evaluation step (Section 3.4), with direct nonuniform sums
# --------------------------------------------------------------------------
def nudft_type2(c, lo1, lo2, y1, y2):
    """g(y) = sum_k c[k] exp(2 pi i y.k), k = (lo1 + i, lo2 + j) over the array c."""
    k1 = lo1 + np.arange(c.shape[0])
    k2 = lo2 + np.arange(c.shape[1])
    E1 = np.exp(2j * np.pi * np.outer(np.asarray(y1) % 1.0, k1))
    E2 = np.exp(2j * np.pi * np.outer(np.asarray(y2) % 1.0, k2))
    return np.einsum("si,ij,sj->s", E1, c, E2)


def stepwise_apply(N, kind, p, fhat, ids, thetas, xidx, eps, rng, r0=48, return_parts=False):
    """The evaluation algorithm step by step, with NUFFTs replaced by direct sums.

    For each wedge ell: separate exp(2 pi i Phi_ell) ~ U T on X x W_ell;
    form fhat_lt = T[t] * fhat on W_ell; g_lt(x) = sum_xi exp(2 pi i y_ell(x).xi)
    fhat_lt(xi) at y_ell(x) = grad_xi Phi(x, xi_hat_ell); then
    u(x) = (1/N) sum_ell sum_t U[x, t] g_lt(x).
    Returns u at xidx (and per-wedge partials and ranks if requested).
    """
    fh = np.asarray(fhat, dtype=np.complex128).reshape(N * N)
    idv = np.asarray(ids).reshape(N * N)
    k1a, k2a = grid_xi(N)
    x1, x2 = x_of_index(N, xidx)
    xidx = np.asarray(xidx, dtype=np.int64)
    u = np.zeros(xidx.size, dtype=np.complex128)
    parts, ranks = [], []
    for ell, th in enumerate(thetas):
        sel = np.nonzero(idv == ell)[0]
        if sel.size == 0:
            parts.append(np.zeros_like(u))
            ranks.append(0)
            continue
        k1, k2 = k1a[sel], k2a[sel]
        sep = randomized_separation(N, kind, p, th, k1, k2, eps, rng, r0=r0)
        y1, y2 = warp(kind, p, x1, x2, th)
        E = _expi(np.outer(y1, k1) + np.outer(y2, k2))       # exp(2 pi i y.xi)
        G = E @ (sep["T"] * fh[sel][None, :]).T                # g_lt(x), (s, q)
        part = np.sum(sep["U"][xidx] * G, axis=1) / N
        u += part
        parts.append(part)
        ranks.append(sep["q"])
    if return_parts:
        return u, parts, ranks
    return u


def rel_l2(approx, exact):
    """Relative l2 error over sample points (Section 4, evaluation error)."""
    approx = np.asarray(approx).ravel()
    exact = np.asarray(exact).ravel()
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
