"""The deterministic factors of Section 3.1 (FIO_FACTORS_TAYLOR) on the GPU.

The library expands each wedge's residual phase in a polar Taylor series,
the exponential of every order in a truncated series, and compresses the
products by QR and SVD.  These tests check (i) the stored factors against the
oracle's exact residual kernel exp(2 pi i Phi_ell) on sampled rows and
columns, (ii) whole applies against the oracle's FP64 direct sum, (iii) the
agreement of Taylor and randomized plans on one input (the cross-check the
deterministic construction provides), and (iv) its error paths.
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


def _apply(plan, fhat, precision="f32"):
    dt = torch.complex128 if precision == "f64" else torch.complex64
    u = plan.apply(torch.from_numpy(np.ascontiguousarray(fhat)).to(dt).cuda())
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.complex128)


# the paper's ellipse family has a/b down to 1/9: its residual phase is
# singular about 0.11 rad off the real angle, so its wedges must be narrower
@pytest.mark.parametrize("N,kind,params,tol,L", [
    (128, "c1c2", (1.0,), 1e-4, 0),
    (128, "paper_ellipse", (1.0,), 1e-4, 64),
    (96, "radial", (0.05, 0.5), 1e-4, 0),
])
def test_taylor_factors_reproduce_residual_kernel(N, kind, params, tol, L):
    p = _plan(N, kind, params, tol, factor_mode="taylor", n_wedges=L)
    assert p.info()["factor_mode"] == 4
    ids = p.wedge_map().ravel()
    k1, k2 = ref.grid_xi(N)
    rng = np.random.default_rng(12)
    for ell in range(0, p.L, 3):
        th = p.wedge_info(ell)["theta"]
        members = np.nonzero(ids == ell)[0]
        G = fi.sample_points(N, 300, rng)
        D = np.sort(rng.choice(members, size=min(300, members.size), replace=False))
        gx, gxi = p.wedge_factors(ell, G, D)
        A = ref.residual_matrix(N, ref.KINDS[kind], params, th, G, k1[D], k2[D])
        err = np.linalg.norm(A - gx @ gxi.T) / np.linalg.norm(A)
        print("  wedge %d rank %d err %.2e" % (ell, gx.shape[1], err))
        assert err < tol, (ell, err)


@pytest.mark.parametrize("N,kind,params,tol,precision,L", [
    (64, "c1c2", (1.0,), 1e-4, "f32", 0),
    (66, "wave", (0.3,), 1e-4, "f32", 0),
    (64, "paper_ellipse", (1.0,), 1e-3, "f32", 64),
    (64, "paper_circle", (1.0,), 1e-3, "f32", 0),
    (64, "c1c2", (1.0,), 1e-6, "f64", 0),
])
def test_taylor_apply_matches_direct_sum(N, kind, params, tol, precision, L):
    rng = np.random.default_rng(13)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    p = _plan(N, kind, params, tol, factor_mode="taylor", precision=precision, n_wedges=L)
    u = _apply(p, fh, precision).ravel()
    exact = od.direct(N, ref.KINDS[kind], params, fh, np.arange(N * N))
    err = ref.rel_l2(u, exact)
    print("  rel-l2 %.3e, ranks %s" % (err, [p.wedge_info(l)["rank"] for l in range(p.L)]))
    assert err <= tol


def test_taylor_and_randomized_plans_agree():
    """The deterministic and the randomized separations approximate one
    operator: their applies agree to the tolerance, both meet it against the
    oracle, and the compressed Taylor ranks stay near the randomized
    (near-optimal) ones."""
    N, tol = 256, 1e-4
    rng = fi.rng_for(14, N)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    pt = _plan(N, "c1c2", (1.0,), tol, factor_mode="taylor")
    pr = _plan(N, "c1c2", (1.0,), tol, factor_mode="stored")
    ut, ur = _apply(pt, fh).ravel(), _apply(pr, fh).ravel()
    xs = fi.sample_points(N, 2048, rng)
    exact = od.direct(N, 2, (1.0,), fh, xs)
    et, er = ref.rel_l2(ut[xs], exact), ref.rel_l2(ur[xs], exact)
    rt = [pt.wedge_info(l)["rank"] for l in range(pt.L)]
    rr = [pr.wedge_info(l)["rank"] for l in range(pr.L)]
    print("  taylor %.2e ranks %s\n  randomized %.2e ranks %s" % (et, rt, er, rr))
    assert et <= tol and er <= tol
    assert ref.rel_l2(ut, ur) <= 2 * tol
    assert sum(rt) <= 1.5 * sum(rr) + len(rr)


def test_taylor_linear_phase_is_rank_one_and_shifts():
    """Phi = x.xi + p.xi: the residual phase vanishes, every wedge has rank
    one, and u is f shifted by p N grid cells."""
    N = 96
    rng = np.random.default_rng(15)
    f = fi.complex_gaussian(N, rng)
    p = _plan(N, "linear", (5 / N, -11 / N), 1e-4, factor_mode="taylor")
    assert all(p.wedge_info(l)["rank"] == 1 for l in range(p.L))
    u = _apply(p, fi.fhat_from_f(f))
    assert ref.rel_l2(u, np.roll(f, (-5, 11), axis=(0, 1))) < 1e-4


def test_taylor_error_paths(tmp_path):
    from paper_math_0610051_amd.fio import FioError
    with pytest.raises(FioError) as e:
        _plan(64, "paper_circle", (1.0,), 1e-3, factor_mode="taylor", amplitude="bessel")
    assert e.value.status == -5
    p = _plan(64, "c1c2", (1.0,), 1e-4, factor_mode="taylor")
    with pytest.raises(FioError) as e:
        p.save(str(tmp_path / "t.plan"))
    assert e.value.status == -5
    # wedges wider than the polar series' radius of convergence (16 wedges
    # reach 0.196 rad; the family's nearest singularity is 0.11 rad away)
    with pytest.raises(FioError) as e:
        _plan(128, "paper_ellipse", (1.0,), 1e-4, factor_mode="taylor", n_wedges=16)
    assert e.value.status == -4 and "converges within" in str(e.value)
