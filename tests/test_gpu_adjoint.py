"""The adjoint apply (Section 3.5) on the GPU against the FP64 adjoint oracle.

fio_apply_adjoint computes the Fourier coefficients of L*g on Omega from a
grid g on X with the forward plan's wedges and factors (type-1 NUFFT).  It
must (i) be the adjoint of the computed forward map up to FP32 rounding,
<L fhat, g> = <fhat, L* g>; (ii) match the oracle's direct sum
hhat(xi) = (1/N) sum_y exp(-2 pi i Phi(y, xi)) g(y) to the plan's tolerance
(relative l2), on whole grids for small N and on sampled frequencies for
large N; (iii) invert a unitary multiplier (L* L = I for x-independent h).
"""
import numpy as np
import pytest

import fio_inputs as fi
from oracle import direct as od
from oracle import reference as ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    od.build(force=False)


def _plan(N, kind, params, tol, **kw):
    from paper_math_0610051_amd import Plan
    print("plan N=%d %s %s tol=%g %s" % (N, kind, params, tol, kw), flush=True)
    return Plan(N, kind, tol, params=params, **kw)


def _dev(a, precision="f32"):
    dt = torch.complex128 if precision == "f64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def _adjoint(plan, g, precision="f32"):
    h = plan.apply_adjoint(_dev(g, precision))
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("N,kind,params,tol,precision", [
    (64, "c1c2", (1.0,), 1e-4, "f32"),
    (66, "radial", (0.05, 0.5), 1e-4, "f32"),
    (64, "paper_ellipse", (1.0,), 1e-3, "f32"),
    (64, "c1c2", (1.0,), 1e-6, "f64"),
])
def test_adjoint_full_grid_matches_direct_sum(N, kind, params, tol, precision):
    rng = np.random.default_rng(41)
    g = fi.complex_gaussian(N, rng)
    p = _plan(N, kind, params, tol, precision=precision)
    h = _adjoint(p, g, precision).ravel()
    exact = od.direct_adjoint(N, ref.KINDS[kind], params, g, np.arange(N * N))
    err = ref.rel_l2(h, exact)
    print("  adjoint rel-l2 %.3e" % err)
    assert err <= tol


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-6)])
def test_adjoint_identity_with_computed_forward(precision, tol):
    """<L~ fhat, g> = <fhat, L~* g> for the computed maps, to rounding."""
    N = 128
    rng = np.random.default_rng(42)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    g = fi.complex_gaussian(N, rng)
    p = _plan(N, "c1c2", (1.1,), tol, precision=precision)
    u = p.apply(_dev(fh, precision))
    torch.cuda.synchronize()
    u = u.cpu().numpy().astype(np.complex128).ravel()
    h = _adjoint(p, g, precision).ravel()
    lhs = np.vdot(g.ravel(), u)
    rhs = np.vdot(h, fh.ravel())
    rel = abs(lhs - rhs) / (np.linalg.norm(g) * np.linalg.norm(fh))
    print("  <Lf,g> - <f,L*g>: %.2e (relative to |f||g|)" % rel)
    assert rel < (2e-6 if precision == "f32" else 1e-13)


def test_adjoint_inverts_a_wave_multiplier():
    """x-independent h: L is unitary, so L* L fhat = fhat to the tolerance."""
    N = 96
    rng = np.random.default_rng(43)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    p = _plan(N, "wave", (0.07,), 1e-4)
    u = p.apply(_dev(fh))
    back = p.apply_adjoint(u)
    torch.cuda.synchronize()
    err = ref.rel_l2(back.cpu().numpy().astype(np.complex128), fh)
    print("  |L*L f - f| / |f| = %.2e" % err)
    assert err < 2e-4


@pytest.mark.parametrize("mode", ["stored", "regen"])
def test_adjoint_batch_and_factor_modes(mode):
    """A batch of right-hand sides equals single applies to rounding (rank
    chunks of the row stage may be summed in another order), and regenerated
    factors agree with stored ones."""
    N, B = 96, 3
    rng = np.random.default_rng(44)
    g = fi.complex_gaussian(N, rng, B=B)
    p = _plan(N, "c1c2", (0.9,), 1e-4, factor_mode=mode, seed=5, max_batch=2)
    hb = _adjoint(p, g).reshape(B, N * N)
    exact = od.direct_adjoint(N, 2, (0.9,), g, np.arange(N * N))
    for b in range(B):
        hs = _adjoint(p, g[b]).ravel()
        assert ref.rel_l2(hb[b], hs) < 1e-6
        assert ref.rel_l2(hb[b], exact[b]) <= 1e-4


@pytest.mark.parametrize("N,B,ns", [(256, 2, 4096), (1024, 2, 1024)])
def test_adjoint_large_sizes_sampled(N, B, ns):
    rng = fi.rng_for(5, N)
    g = fi.complex_gaussian(N, rng, B=B)
    p = _plan(N, "c1c2", (1.0,), 1e-4, max_batch=B)
    h = _adjoint(p, g).reshape(B, N * N)
    ks = fi.sample_points(N, ns, rng)
    print("  oracle: %d frequencies x %d inputs" % (ns, B), flush=True)
    exact = od.direct_adjoint(N, 2, (1.0,), g, ks)
    for b in range(B):
        err = ref.rel_l2(h[b, ks], exact[b])
        print("  N=%d input %d rel-l2 %.3e" % (N, b, err))
        assert err <= 1e-4


def test_adjoint_paper_circles_composition():
    """The composition L* L of the paper's last example (phase x.xi + r(x)|xi|
    with the circles of eq. (circlerad)) against the oracle's two direct sums."""
    N = 64
    rng = np.random.default_rng(45)
    f = fi.complex_gaussian(N, rng)
    fh = fi.fhat_from_f(f)
    p = _plan(N, "paper_circle", (1.0,), 1e-3)
    u = p.apply(_dev(fh))
    back = p.apply_adjoint(u)
    torch.cuda.synchronize()
    got = back.cpu().numpy().astype(np.complex128).ravel()
    u_ref = od.direct(N, 5, (1.0,), fh, np.arange(N * N)).reshape(N, N)
    want = od.direct_adjoint(N, 5, (1.0,), u_ref, np.arange(N * N))
    err = ref.rel_l2(got, want)
    print("  L*L rel-l2 %.3e" % err)
    assert err <= 2e-3
