"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every check calls the library through its ctypes binding and compares with
oracle/ on the same seeded inputs.  Integer work (the wedge partition) must
agree bit for bit; floating-point results must meet the relative l2
tolerance the plan was built for (default 1e-4), as the paper measures
errors (Section 4).  Element-wise maxima are also bounded.
"""
import math

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
    from paper_math_0610051_amd import fio  # noqa: F401  (raises if the library is missing)


def _plan(N, kind, params, tol, **kw):
    from paper_math_0610051_amd import Plan
    print("plan N=%d %s %s tol=%g %s" % (N, kind, params, tol, kw), flush=True)
    return Plan(N, kind, tol, params=params, **kw)


def _dev(a, precision="f32"):
    dt = torch.complex128 if precision == "f64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def _apply(plan, fhat, precision="f32"):
    u = plan.apply(_dev(fhat, precision))
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.complex128)


# ------------------------------------------------------------------ a2: partition (integer, bit-exact)
@pytest.mark.parametrize("N,partition,L", [(64, "equiangular", 0), (256, "equiangular", 0), (100, "equiangular", 24),
                                           (64, "coronae", 0), (256, "coronae", 0)])
def test_wedge_map_bit_exact(N, partition, L):
    p = _plan(N, "c1c2", (1.0,), 1e-2, partition=partition, n_wedges=L)
    if partition == "coronae":
        ids, th = ref.corona_partition(N)
    else:
        ids, th = ref.equiangular_partition(N, L or 8 * math.ceil(math.sqrt(N) / 8))
    assert np.array_equal(p.wedge_map(), ids)
    assert p.L == len(th)
    for ell in range(p.L):
        assert abs(p.wedge_info(ell)["theta"] - th[ell]) < 1e-15


def test_wedge_boxes_hold_their_sheared_members():
    N = 128
    p = _plan(N, "c1c2", (1.0,), 1e-2)
    ids = p.wedge_map().ravel()
    k1, k2 = ref.grid_xi(N)
    for ell in range(p.L):
        w = p.wedge_info(ell)
        M = np.array(w["M"]).reshape(2, 2)
        assert abs(round(np.linalg.det(M))) == 1
        sel = ids == ell
        a = M @ np.stack([k1[sel], k2[sel]]) - np.array(w["xi_c"])[:, None]
        for d in range(2):
            # the box is the sheared members' bounding box, centred: tight on both sides
            assert a[d].min() == w["lo"][d] and a[d].max() == w["lo"][d] + w["box"][d] - 1
            assert w["fine"][d] >= 2 * w["box"][d]
        assert w["box"][0] >= w["box"][1]  # axis 1 is the long side


# ------------------------------------------------------------------ a3: warped points (FP64)
@pytest.mark.parametrize("kind,params", [("c1c2", (1.3,)), ("radial", (0.05, 0.5)), ("paper_ellipse", (1.0,))])
def test_warped_points_fp64(kind, params):
    N = 256
    p = _plan(N, kind, params, 1e-2)
    rng = np.random.default_rng(1)
    xs = fi.sample_points(N, 500, rng)
    x1, x2 = ref.x_of_index(N, xs)
    for ell in (0, 3, p.L - 1):
        th = p.wedge_info(ell)["theta"]
        y = p.wedge_warp(ell, xs)
        e1, e2 = ref.warp(ref.KINDS[kind], params, x1, x2, th)
        assert np.max(np.abs(y[:, 0] - e1)) < 1e-13 and np.max(np.abs(y[:, 1] - e2)) < 1e-13


# ------------------------------------------------------------------ a4: separated factors vs exp(2 pi i Phi_ell)
@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-6)])
def test_stored_factors_reproduce_residual_kernel(precision, tol):
    """Independent s x s estimate (Section 4) of the stored factors against the oracle's A."""
    N = 128
    p = _plan(N, "c1c2", (1.0,), tol, precision=precision)
    ids = p.wedge_map().ravel()
    k1, k2 = ref.grid_xi(N)
    rng = np.random.default_rng(2)
    for ell in range(0, p.L, 3):
        th = p.wedge_info(ell)["theta"]
        members = np.nonzero(ids == ell)[0]
        G = fi.sample_points(N, 200, rng)
        D = np.sort(rng.choice(members, size=min(200, members.size), replace=False))
        gx, gxi = p.wedge_factors(ell, G, D)
        A = ref.residual_matrix(N, 2, (1.0,), th, G, k1[D], k2[D])
        err = np.linalg.norm(A - gx @ gxi.T) / np.linalg.norm(A)
        assert err < tol, (ell, err)


# ------------------------------------------------------------------ closed forms through the fast path
@pytest.mark.parametrize("N", [64, 130])
def test_identity_phase_returns_input(N):
    """Phi = x.xi: u = f (rank 1, so only NUFFT and FP32 error remain)."""
    rng = np.random.default_rng(3)
    f = fi.complex_gaussian(N, rng)
    p = _plan(N, "linear", (0.0, 0.0), 1e-4)
    u = _apply(p, fi.fhat_from_f(f))
    assert ref.rel_l2(u, f) < 1e-4
    assert np.max(np.abs(u - f)) < 1e-4 * np.max(np.abs(f)) * 5


def test_grid_shift_is_a_roll():
    N = 96
    rng = np.random.default_rng(4)
    f = fi.complex_gaussian(N, rng)
    p = _plan(N, "linear", (5 / N, -11 / N), 1e-4)
    u = _apply(p, fi.fhat_from_f(f))
    assert ref.rel_l2(u, np.roll(f, (-5, 11), axis=(0, 1))) < 1e-4


@pytest.mark.parametrize("ct", [0.05, -0.12])
def test_wave_multiplier_closed_form(ct):
    N = 128
    rng = np.random.default_rng(5)
    f = fi.complex_gaussian(N, rng)
    p = _plan(N, "wave", (ct,), 1e-4)
    u = _apply(p, fi.fhat_from_f(f))
    expect = ref.multiplier_solution(N, lambda a, b: ref.h(1, (ct,), 0.0, 0.0, a, b), f)
    assert ref.rel_l2(u, expect) < 1e-4


# ------------------------------------------------------------------ end to end vs the direct sum
@pytest.mark.parametrize("N,kind,params,tol,precision", [
    (64, "c1c2", (1.0,), 1e-4, "f32"),
    (64, "radial", (0.05, 0.5), 1e-4, "f32"),
    (66, "c1c2", (1.2,), 1e-4, "f32"),
    (64, "paper_ellipse", (1.0,), 1e-3, "f32"),
    (64, "paper_circle", (1.0,), 1e-3, "f32"),
    (64, "c1c2", (1.0,), 1e-6, "f64"),
    (128, "c1c2", (1.0,), 1e-2, "f32"),
])
def test_full_grid_matches_direct_sum(N, kind, params, tol, precision):
    """Every output point against the FP64 direct sum (A28 relative l2 <= tol)."""
    rng = np.random.default_rng(6)
    f = fi.complex_gaussian(N, rng)
    fhat = fi.fhat_from_f(f)
    p = _plan(N, kind, params, tol, precision=precision)
    u = _apply(p, fhat, precision).ravel()
    exact = od.direct(N, ref.KINDS[kind], params, fhat, np.arange(N * N))
    err = ref.rel_l2(u, exact)
    print("  rel-l2 %.3e  max-abs/max %.3e" % (err, np.max(np.abs(u - exact)) / np.max(np.abs(exact))))
    assert err <= tol
    assert np.max(np.abs(u - exact)) <= 10 * tol * np.max(np.abs(exact))


def test_small_config_fp64_coronae_full_direct_sum():
    """N = 64, real white noise, c1/c2 phase, dyadic coronae, FP64, 1e-6 on all 4096 points."""
    N = 64
    f = fi.white_noise_real(N, fi.rng_for(0))
    fhat = fi.fhat_from_f(f)
    p = _plan(N, "c1c2", (1.0,), 1e-6, precision="f64", partition="coronae")
    u = _apply(p, fhat, "f64").ravel()
    exact = od.direct(N, 2, (1.0,), fhat, np.arange(N * N))
    assert ref.rel_l2(u, exact) <= 1e-6


_N256_EXACT = {}


def _n256_case(kind, params):
    """N = 256 complex-Gaussian input of one family and its direct sum at all
    65536 outputs (computed once per family and shared by the tolerances)."""
    if kind not in _N256_EXACT:
        N = 256
        rng = fi.rng_for(1, 0)
        fhat = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=2))
        print("  oracle: all %d outputs x 2 inputs, %s" % (N * N, kind), flush=True)
        _N256_EXACT[kind] = (fhat, od.direct(N, ref.KINDS[kind], params, fhat, np.arange(N * N)))
    return _N256_EXACT[kind]


@pytest.mark.parametrize("kind,params", [("c1c2", (1.0,)), ("radial", (0.05, 0.5))])
@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_n256_tolerance_sweep_all_points(kind, params, tol):
    """N = 256, complex Gaussian f, FP32 data with FP64 phase, against the
    direct sum at all 65536 outputs, per input (two inputs)."""
    N = 256
    fhat, exact = _n256_case(kind, params)
    p = _plan(N, kind, params, tol)
    u = _apply(p, fhat).reshape(2, N * N)
    for b in range(2):
        err = ref.rel_l2(u[b], exact[b])
        print("  input %d rel-l2 %.3e ranks %d..%d" % (b, err, p.info()["min_rank"], p.info()["max_rank"]))
        assert err <= tol


# ------------------------------------------------------------------ per wedge (Section 1.3 partition of unity)
def test_per_wedge_partials_match_direct_sums():
    N = 64
    rng = np.random.default_rng(7)
    fhat = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    p = _plan(N, "c1c2", (1.0,), 1e-5)
    ids = p.wedge_map()
    xs = np.arange(N * N)
    fd = _dev(fhat)
    total = np.zeros(N * N, complex)
    for ell in range(p.L):
        part = p.apply_wedges(ell, ell + 1, fd)
        torch.cuda.synchronize()
        part = part.cpu().numpy().ravel().astype(complex)
        exact = od.direct(N, 2, (1.0,), fhat, xs, member=ids, only=ell)
        assert ref.rel_l2(part, exact) < 2e-4, ell
        total += part
    full = _apply(p, fhat).ravel()
    assert ref.rel_l2(total, full) < 1e-6


# ------------------------------------------------------------------ batching, determinism, multi-instance
def test_batch_is_bitwise_a_loop_of_singles():
    N = 128
    rng = np.random.default_rng(8)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=6))
    p = _plan(N, "c1c2", (1.0,), 1e-4, max_batch=4)
    ub = p.apply(_dev(fh))
    torch.cuda.synchronize()
    ub = ub.cpu().numpy()
    for b in range(6):
        us = _apply(p, fh[b])
        assert np.array_equal(ub[b].astype(np.complex128), us)


def test_apply_is_deterministic():
    N = 64
    fh = fi.fhat_from_f(fi.complex_gaussian(N, np.random.default_rng(9)))
    p = _plan(N, "radial", (0.05, 0.5), 1e-4)
    a = _apply(p, fh)
    b = _apply(p, fh)
    assert np.array_equal(a, b)


def test_multi_instance_matches_singles():
    from paper_math_0610051_amd import apply_multi
    rng = np.random.default_rng(10)
    specs = [(64, "c1c2", (0.7,), 2), (128, "radial", (0.05, 0.5), 1), (96, "c1c2", (1.4,), 3)]
    plans, fh = [], []
    for N, kind, params, B in specs:
        plans.append(_plan(N, kind, params, 1e-4))
        fh.append(_dev(fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))))
    outs = apply_multi(plans, fh)
    torch.cuda.synchronize()
    for p, f, u in zip(plans, fh, outs):
        single = p.apply(f)
        torch.cuda.synchronize()
        assert torch.equal(single, u)


# ------------------------------------------------------------------ large sizes, sampled outputs
@pytest.mark.parametrize("N,B", [(512, 2), (1024, 1)])
def test_large_sizes_sampled(N, B):
    rng = fi.rng_for(2, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    xs = fi.sample_points(N, 384, rng)
    p = _plan(N, "c1c2", (1.0,), 1e-4)
    u = p.apply(_dev(fh))
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(B, N * N)[:, xs]
    exact = od.direct(N, 2, (1.0,), fh, xs)
    err = ref.rel_l2(u, exact)
    print("  N=%d rel-l2 %.3e" % (N, err))
    assert err <= 1e-4


@pytest.mark.parametrize("sigma", [1.5, 2.5])
def test_other_oversampling_factors_full_grid(sigma):
    """Oversampling other than 2: below 2 a box fills more than half of its
    grid rows (the row stage then looks up part of its cells per right-hand
    side); above 2 the grids grow.  Both must meet the tolerance."""
    N, tol = 128, 1e-3
    rng = fi.rng_for(1, 3)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=2))
    p = _plan(N, "c1c2", (1.0,), tol, sigma=sigma)
    u = p.apply(_dev(fh))
    torch.cuda.synchronize()
    u = u.cpu().numpy().astype(np.complex128).reshape(2, N * N)
    exact = od.direct(N, 2, (1.0,), fh, np.arange(N * N))
    err = ref.rel_l2(u, exact)
    print("  sigma %.2f: kernel width %d, rel-l2 %.3e" % (sigma, p.info()["kernel_width"], err))
    assert err <= tol


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_regenerated_factors_match_stored_ones(precision):
    """FIO_FACTORS_REGEN keeps only the compressed factors (sampled columns and
    Z = V S^-1), reduced to the columns an interpolative decomposition keeps
    (far below the separation threshold), and recomputes gamma^x in the
    apply.  With the same seed the separation is the same, so the apply must
    agree with the stored-factor plan far inside the tolerance, meet the
    tolerance, and hold far fewer factor bytes."""
    N, tol = 128, 1e-4
    rng = fi.rng_for(1, 5)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=3))
    ps = _plan(N, "c1c2", (1.0,), tol, precision=precision, factor_mode="stored", seed=77)
    pr = _plan(N, "c1c2", (1.0,), tol, precision=precision, factor_mode="regen", seed=77)
    assert pr.info()["factor_mode"] == 2
    us = _apply(ps, fh, precision).reshape(3, N * N)
    ur = _apply(pr, fh, precision).reshape(3, N * N)
    diff = ref.rel_l2(ur, us)
    exact = od.direct(N, 2, (1.0,), fh, np.arange(N * N))
    err = ref.rel_l2(ur, exact)
    fs, fr = ps.info()["factor_bytes"], pr.info()["factor_bytes"]
    print("  %s: regen vs stored %.2e, regen vs direct %.2e, factor bytes %d -> %d"
          % (precision, diff, err, fs, fr))
    assert diff < 0.02 * tol
    assert err <= tol
    assert fr * 4 < fs
    # the exported spatial factors agree: host FP64 regeneration from the
    # kept columns against the stored ones from all sampled columns; their
    # difference is the decomposition's, which the sum with Z ~ 1/s_q scales
    # up in the weakest factors (whose gamma^xi are small: the applies above
    # differ by 2e-7)
    xs = np.arange(0, N * N, 97)
    for ell in (0, pr.L // 3):
        gr, _ = pr.wedge_factors(ell, xs)
        gs, _ = ps.wedge_factors(ell, xs)
        rel = np.linalg.norm(gr - gs) / np.linalg.norm(gs)
        print("  wedge %d: spatial factors differ by %.2e" % (ell, rel))
        assert rel <= tol


def test_fp64_long_columns_in_rank_chunks():
    """FP64 at a tight tolerance: when a grid column of all ranks exceeds the
    LDS transform buffer (n1 * qpad > 4096 complex doubles), the column stage
    transforms it in rank chunks.  The result must still meet the tolerance."""
    N, tol = 512, 1e-6
    rng = fi.rng_for(1, 7)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    xs = fi.sample_points(N, 512, rng)
    p = _plan(N, "c1c2", (1.0,), tol, precision="f64")
    chunked = 0
    for ell in range(p.L):
        wi = p.wedge_info(ell)
        qpad = wi["rank"] + (wi["rank"] & 1)
        chunked += wi["rank"] > 0 and wi["fine"][0] * qpad > 4096
    print("  wedges with rank-chunked columns: %d of %d; %s" % (chunked, p.L, p.info()))
    assert chunked > 0
    u = _apply(p, fh, "f64").ravel()[xs]
    exact = od.direct(N, 2, (1.0,), fh, xs)
    err = ref.rel_l2(u, exact)
    print("  rel-l2 %.3e" % err)
    assert err <= tol


def test_batch_of_64_in_one_graph_at_512():
    """64 complex-Gaussian right-hand sides at N = 512 in one fused graph
    launch (all wedges, all right-hand sides): every input meets the budget
    at sampled points, and the result equals the plain batched apply."""
    from paper_math_0610051_amd import apply_multi
    N, B, tol = 512, 64, 1e-4
    rng = fi.rng_for(2, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    xs = fi.sample_points(N, 2048, rng)
    p = _plan(N, "c1c2", (1.0,), tol, max_batch=B)
    fd = _dev(fh)
    u = apply_multi([p], [fd])[0]
    ub = p.apply(fd)
    torch.cuda.synchronize()
    assert torch.equal(u, ub)
    got = u.cpu().numpy().astype(np.complex128).reshape(B, N * N)[:, xs]
    exact = od.direct(N, 2, (1.0,), fh, xs)
    errs = [ref.rel_l2(got[b], exact[b]) for b in range(B)]
    print("  worst of %d inputs: rel-l2 %.3e" % (B, max(errs)))
    assert max(errs) <= tol


# ------------------------------------------------------------------ fused multi-instance launch (HIP graph)
def test_multi_graph_replays_match_eager_results():
    """The captured graph is replayed several times with eager work in between;
    every replay must equal the eager single-plan results bit for bit."""
    from paper_math_0610051_amd import apply_multi
    rng = np.random.default_rng(11)
    specs = [(64, "c1c2", (1.1,), 2), (80, "radial", (0.05, 0.5), 1)]
    plans = [_plan(N, k, pr, 1e-4) for N, k, pr, _ in specs]
    fh = [_dev(fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))) for N, _, _, B in specs]
    eager = []
    for p, f in zip(plans, fh):
        eager.append(p.apply(f).clone())
    torch.cuda.synchronize()
    outs = [torch.empty_like(f) for f in fh]
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        apply_multi(plans, fh, outs)
        torch.cuda.synchronize()
        junk = plans[0].apply(fh[0])  # eager work between replays
        torch.cuda.synchronize()
        del junk
        for e, o in zip(eager, outs):
            assert torch.equal(e, o), rep
    # new output buffers refresh the argument table of the cached graph
    outs2 = apply_multi(plans, fh)
    torch.cuda.synchronize()
    for e, o in zip(eager, outs2):
        assert torch.equal(e, o)


def test_uneven_batch_against_direct_sums():
    """32 instances, N in {128, 256, 512, 1024}, c1/c2 (scale in [0.5, 1.5]) or rho(x)|xi|,
    complex Gaussian or 20 Gaussian bumps; one fused launch; per-instance relative l2
    error on 2048 sampled outputs (all outputs for N <= 256)."""
    from paper_math_0610051_amd import apply_multi
    insts = fi.uneven_instances(32, seed=3000)
    plans, fh, samples = [], [], []
    for inst in insts:
        kind, params = ("c1c2", (inst["scale"],)) if inst["family"] == "c1c2" else ("radial", (0.05, 0.5))
        plans.append(_plan(inst["N"], kind, params, 1e-4))
        fhat = fi.fhat_from_f(fi.instance_field(inst))
        fh.append(fhat)
        # 2048 sampled outputs per instance, every output when N <= 256
        n = inst["N"]
        samples.append(np.arange(n * n) if n <= 256 else fi.sample_points(n, 2048, np.random.default_rng(inst["seed"] + 7)))
    dev = [_dev(f) for f in fh]
    outs = apply_multi(plans, dev)
    torch.cuda.synchronize()
    worst = 0.0
    for inst, p, f, o, xs in zip(insts, plans, fh, outs, samples):
        kind = 2 if inst["family"] == "c1c2" else 3
        params = (inst["scale"],) if kind == 2 else (0.05, 0.5)
        exact = od.direct(inst["N"], kind, params, f, xs)
        got = o.cpu().numpy().ravel()[xs]
        err = ref.rel_l2(got, exact)
        worst = max(worst, err)
        assert err <= 1e-4, (inst, err)
    print("  worst per-instance rel-l2 %.3e" % worst)


# ------------------------------------------------------------------ on-device probe and autotuner
def test_device_probe_agrees_with_cpu_oracle():
    """fio_probe_error against u taken from the CPU oracle: ~0 for the exact u and the
    planted relative perturbation level for a perturbed one."""
    N = 32
    rng = np.random.default_rng(12)
    fhat = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    p = _plan(N, "c1c2", (1.0,), 1e-4, precision="f64")
    exact = od.direct(N, 2, (1.0,), fhat, np.arange(N * N)).reshape(N, N)
    fd = _dev(fhat, "f64")
    assert p.probe_error(fd, _dev(exact, "f64"), nsamples=256) < 1e-12
    noise = fi.complex_gaussian(N, rng)
    pert = exact + 1e-3 * noise * np.linalg.norm(exact) / np.linalg.norm(noise)
    e = p.probe_error(fd, _dev(pert, "f64"), nsamples=1024)
    assert 0.7e-3 < e < 1.3e-3


def test_autotuner_choice_meets_the_budget():
    from paper_math_0610051_amd import autotune
    N, tol = 128, 1e-4
    best, tried = autotune(N, "c1c2", tol, params=(1.0,), B=2)
    print("  tried %d, best %s" % (len(tried), best))
    assert len(tried) >= 8 and best["error"] <= 0.8 * tol
    assert best["ms_per_rhs"] == min(t["ms_per_rhs"] for t in tried if t["error"] <= 0.8 * tol)
    rng = np.random.default_rng(13)
    fhat = fi.fhat_from_f(fi.complex_gaussian(N, rng))
    p = _plan(N, "c1c2", (1.0,), tol, n_wedges=best["n_wedges"], sigma=best["sigma"],
              sep_tol_frac=best["sep_tol_frac"], nufft_tol_frac=best["nufft_tol_frac"],
              kernel_width=best["kernel_width"])
    assert p.info()["kernel_width"] == best["kernel_width"]
    u = _apply(p, fhat).ravel()
    xs = fi.sample_points(N, 1024, rng)
    assert ref.rel_l2(u[xs], od.direct(N, 2, (1.0,), fhat, xs)) <= tol


@pytest.mark.parametrize("precision,mode", [("f32", "stored"), ("f32", "regen"), ("f64", "stored")])
def test_saved_plan_applies_bit_for_bit(tmp_path, precision, mode):
    """fio_plan_save / fio_plan_load: the loaded plan rebuilds the geometry and
    the factors from the saved compressed separation and must apply exactly
    like the saved plan; a corrupted file is refused."""
    from paper_math_0610051_amd import fio
    N, tol = 128, (1e-4 if precision == "f32" else 1e-6)
    rng = fi.rng_for(1, 9)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=2))
    p = _plan(N, "c1c2", (1.0,), tol, precision=precision, factor_mode=mode, seed=321)
    path = tmp_path / "op.plan"
    p.save(path)
    q = fio.Plan.load(path)
    a, b = p.info(), q.info()
    for k in ("N", "L", "precision", "factor_mode", "kernel_width", "min_rank", "max_rank", "fine_cells",
              "box_cells", "factor_bytes"):
        assert a[k] == b[k], k
    assert a["max_sep_error"] == b["max_sep_error"]
    ua = _apply(p, fh, precision)
    ub = _apply(q, fh, precision)
    assert np.array_equal(ua, ub)
    raw = bytearray(path.read_bytes())
    raw[len(raw) // 2] ^= 0xFF
    bad = tmp_path / "bad.plan"
    bad.write_bytes(bytes(raw))
    with pytest.raises(fio.FioError) as e:
        fio.Plan.load(bad)
    assert e.value.status == fio.FIO_EINVAL


def test_benchmark_plan_against_direct_sums():
    """The plan the benchmark times: N = 1024, c1/c2 at scale 1, tol 1e-4,
    L = 40, sigma = 2, tolerance split 0.4 / 0.15, kernel width 5 (one below
    the width bound), B = 8 complex-Gaussian inputs of the benchmark's seed.
    Every input meets the budget on its own at 3072 sampled outputs."""
    N, B, tol = 1024, 8, 1e-4
    rng = fi.rng_for(4, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    p = _plan(N, "c1c2", (1.0,), tol, max_batch=B, n_wedges=40, sigma=2.0, sep_tol_frac=0.4,
              nufft_tol_frac=0.15, kernel_width=5)
    info = p.info()
    assert info["kernel_width"] == 5 and info["L"] == 40
    u = p.apply(_dev(fh))
    torch.cuda.synchronize()
    xs = fi.sample_points(N, 3072, np.random.default_rng(4321))
    got = u.cpu().numpy().astype(np.complex128).reshape(B, N * N)[:, xs]
    print("  oracle: %d outputs x %d inputs" % (xs.size, B), flush=True)
    exact = od.direct(N, 2, (1.0,), fh, xs)
    errs = [ref.rel_l2(got[b], exact[b]) for b in range(B)]
    print("  per-input rel-l2 %s; ranks %d..%d" % (["%.2e" % e for e in errs], info["min_rank"], info["max_rank"]))
    assert max(errs) <= tol


def test_multi_rejects_or_serialises_a_repeated_plan():
    """The same plan twice in one fused call: its workspace cannot hold both
    instances at once, so the result must still equal two separate applies."""
    from paper_math_0610051_amd import apply_multi
    N = 64
    rng = np.random.default_rng(15)
    p = _plan(N, "c1c2", (1.0,), 1e-4)
    f1 = _dev(fi.fhat_from_f(fi.complex_gaussian(N, rng)))
    f2 = _dev(fi.fhat_from_f(fi.complex_gaussian(N, rng)))
    u1, u2 = apply_multi([p, p], [f1, f2])
    torch.cuda.synchronize()
    a1, a2 = p.apply(f1), p.apply(f2)
    torch.cuda.synchronize()
    assert torch.equal(u1, a1) and torch.equal(u2, a2)


def test_multi_mixed_widths_in_one_launch():
    """Instances whose tolerances need different kernel widths share one fused
    launch (the widest stencil, each instance weighting with its own width):
    the result equals each plan's own apply to rounding and meets its budget."""
    from paper_math_0610051_amd import apply_multi
    rng = np.random.default_rng(16)
    specs = [(64, "c1c2", (1.0,), 1e-2, 2), (96, "radial", (0.05, 0.5), 1e-4, 1), (80, "c1c2", (0.8,), 2e-6, 1)]
    plans, fh, host = [], [], []
    for N, kind, params, tol, B in specs:
        plans.append(_plan(N, kind, params, tol))
        h = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
        host.append(h)
        fh.append(_dev(h))
    widths = sorted({p.info()["kernel_width"] for p in plans})
    print("  kernel widths %s" % widths)
    assert len(widths) >= 2
    outs = apply_multi(plans, fh)
    torch.cuda.synchronize()
    for (N, kind, params, tol, B), p, f, h, u in zip(specs, plans, fh, host, outs):
        single = p.apply(f)
        torch.cuda.synchronize()
        a = u.cpu().numpy().astype(np.complex128).reshape(B, N * N)
        b = single.cpu().numpy().astype(np.complex128).reshape(B, N * N)
        assert ref.rel_l2(a, b) < 1e-6
        exact = od.direct(N, ref.KINDS[kind], params, h, np.arange(N * N)).reshape(B, N * N)
        assert ref.rel_l2(a, exact) <= tol
