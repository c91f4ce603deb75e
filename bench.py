"""Benchmark of the FIO apply on one MI355X.

Default workload (one JSON line): N = 1024, B = 8 complex-Gaussian right-hand
sides under the c1/c2 ellipse phase, FP32 data with FP64 phase, tolerance
1e-4 relative l2.  One step = one fio_apply_batch of the 8 right-hand sides
through the whole hot path (window + row FFT, column FFT, interpolate +
combine), inputs resident in device memory.  Wedge count, oversampling and
tolerance split come from the library's autotuner (cached in
$FIO_TUNE_CACHE, default /tmp/fio_tune_cache.txt).

Other workloads (each prints its own JSON line):
  --workload batch512 64 right-hand sides at N = 512 in one fused graph launch
  --workload uneven   32 instances, N in {128, ..., 1024}, one fused launch
  --workload learned  network-factor plan vs exact plan at N = 1024
  --workload paper    the paper's Table 3 / Table 4 examples, N = 64 ... 512
  --workload adjoint  the adjoint L* on the N = 1024 plan, 8 right-hand sides

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0             # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector, published (counts packed FP32 FMAs)
FP32_NONPACKED_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x FMA (2 flop) x 2.4 GHz: the rate without
                                  # packed FP32, which this build disables
STAGES = ("window_rowfft", "colfft", "interp_combine")


from paper_math_0610051_amd import pmc  # noqa: E402


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def stage_work(plan, B):
    """Algorithmic bytes and flops per stage for one apply of B right-hand sides.

    Per wedge (box B1 x B2, grid n1 x n2, rank q, |W| members), complex64 =
    8 bytes; bytes count the rank padded to even (the stored 16-byte rank
    pairs the kernels must move), flops the true rank:
      stage 0 reads fhat on W and gamma^xi (q per member), writes B1 * n2 * q;
      stage 1 reads B1 * n2 * q, writes n1 * n2 * q;
      stage 2 reads n1 * n2 * q and gamma^x (N^2 q, once per launch of up to 8
              right-hand sides), writes N^2 per right-hand side; its flops are
              N^2 q (4 w^2 + 4 w + 8) per wedge and right-hand side (a w x w
              real-weighted stencil of complex values, the w-point weights of
              both axes, and the factor and modulation products).
    """
    info = plan.info()
    N, w = info["N"], info["kernel_width"]
    NN = N * N
    es = 16 if plan.precision == "f64" else 8
    by = [0.0, 0.0, 0.0]
    fl = 0.0
    gx_bytes = 0.0
    for ell in range(info["L"]):
        wi = plan.wedge_info(ell)
        if wi["rank"] == 0:
            continue
        q = wi["rank"] + (wi["rank"] & 1)
        B1, B2 = wi["box"]
        n1, n2 = wi["fine"]
        nm = wi["members"]
        by[0] += es * (nm + nm * q + B1 * n2 * q) * B
        by[1] += es * (B1 * n2 * q + n1 * n2 * q) * B
        by[2] += es * (n1 * n2 * q) * B
        gx_bytes += es * NN * q
        fl += NN * wi["rank"] * (4.0 * w * w + 4.0 * w + 8.0) * B
    by[2] += gx_bytes * math.ceil(B / 8) + es * NN * B
    return by, fl


def cpu_model():
    """Host CPU model name (lscpu's "Model name", else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_check(N, phase_kind, params, fh, samples, seed):
    """FP64 direct-sum oracle at `samples` random outputs of every right-hand
    side (all host threads); returns (sample indices, reference values, seconds, threads)."""
    import numpy as np
    from oracle import direct as od

    od.build(force=False)
    rng = np.random.default_rng(seed)
    xs = np.sort(rng.choice(N * N, size=samples, replace=False))
    t0 = time.perf_counter()
    ref = od.direct(N, phase_kind, params, fh, xs)
    return xs, ref, time.perf_counter() - t0, od.max_threads()


def cpu_baseline(N, phase_kind, params, fh, samples, dt, threads, one_thread_samples):
    """The oracle's throughput, extrapolated to all N^2 outputs, from the timed
    all-thread check and from a smaller run on one thread."""
    import numpy as np
    from oracle import direct as od

    B = fh.shape[0]
    rng = np.random.default_rng(99)
    xs1 = np.sort(rng.choice(N * N, size=one_thread_samples, replace=False))
    t0 = time.perf_counter()
    od.direct(N, phase_kind, params, fh, xs1, threads=1)
    dt1 = time.perf_counter() - t0
    od.direct(N, phase_kind, params, fh[:1], xs1[:1], threads=threads)  # restore the thread count
    return dict(value=B / (dt * (N * N) / samples), unit="applies/s", cores=threads, kind="oracle",
                model=cpu_model(),
                sample="%d random outputs x %d RHS of the N=%d workload (%.2e kernel terms, shared by the RHS) "
                       "in %.1f s on %d threads; extrapolated to all N^2 outputs"
                       % (samples, B, N, float(samples) * N * N, dt, threads),
                one_thread=dict(value=B / (dt1 * (N * N) / one_thread_samples), unit="applies/s", cores=1,
                                sample="%d random outputs x %d RHS in %.1f s on one thread"
                                       % (one_thread_samples, B, dt1)))


def tuned_plan(N, tol, B, fixed=None, factor_mode="auto"):
    """Plan with the autotuner's choice (cached on disk), or with fixed
    (n_wedges, sigma, sep_tol_frac, nufft_tol_frac) when given."""
    from paper_math_0610051_amd import Plan, autotune
    if fixed is None:
        os.environ.setdefault("FIO_TUNE_CACHE", "/tmp/fio_tune_cache.txt")
        t0 = time.perf_counter()
        best, tried = autotune(N, "c1c2", tol, params=(1.0,), B=B)
        log("autotune %.1f s (%d candidates): %s" % (time.perf_counter() - t0, len(tried), best))
    else:
        L, sg, st, nt = fixed[:4]
        best = dict(n_wedges=int(L), sigma=float(sg), sep_tol_frac=float(st), nufft_tol_frac=float(nt),
                    kernel_width=int(fixed[4]) if len(fixed) > 4 else 0)
    t0 = time.perf_counter()
    plan = Plan(N, "c1c2", tol, params=(1.0,), max_batch=B, n_wedges=best["n_wedges"], sigma=best["sigma"],
                sep_tol_frac=best["sep_tol_frac"], nufft_tol_frac=best["nufft_tol_frac"],
                kernel_width=best.get("kernel_width", 0), factor_mode=factor_mode)
    return plan, time.perf_counter() - t0, best


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: read + write bytes of fio_copy per second."""
    import torch
    from paper_math_0610051_amd import copy
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ok = bool(torch.equal(a, b))
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ok


def time_applies(plan, fd, out, steps, warmup, profile=False):
    import torch
    for _ in range(warmup):
        plan.apply(fd, out)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(fd, out)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_batched(args):
    import numpy as np
    import torch

    import fio_inputs as fi

    N, B = args.N, args.batch
    copy_gbs, copy_ok = copy_bandwidth()
    if not copy_ok:
        raise SystemExit("fio_copy produced a wrong copy")
    log("fio_copy: %.0f GB/s (read + write)" % copy_gbs)
    log("N=%d B=%d tol=%g: planning" % (N, B, args.tol))
    fixed = tuple(float(v) for v in args.plan_params.split(",")) if args.plan_params else None
    plan, plan_s, best = tuned_plan(N, args.tol, B, fixed, args.factor_mode)
    info = plan.info()
    rng = fi.rng_for(4, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    fd = torch.from_numpy(fh.astype(np.complex64)).cuda()
    out = torch.empty_like(fd)
    log("plan %.1f s, L=%d ranks %d..%d w=%d sigma=%g; timing" % (plan_s, info["L"], info["min_rank"],
                                                                  info["max_rank"], info["kernel_width"],
                                                                  info["sigma"]))
    elapsed = time_applies(plan, fd, out, args.steps, args.warmup, profile=True)
    ms, launches = plan.profile_read()
    plan.profile(False)
    value = B * args.steps / elapsed
    # the same right-hand sides one apply each (no batching), for comparison
    single_value = None
    if not args.no_compare:
        single = torch.empty_like(fd[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps // 2)):
            for b in range(B):
                plan.apply(fd[b], single)
        torch.cuda.synchronize()
        single_value = B * max(1, args.steps // 2) / (time.perf_counter() - t0)
    by, fl = stage_work(plan, B)
    steps = args.steps
    per_launch_ms = [ms[i] / max(1, launches[i]) for i in range(3)]
    stage_ms = [ms[i] / steps for i in range(3)]
    lps = [launches[i] / steps for i in range(3)]
    dom = int(np.argmax(stage_ms))
    kname = ("k_rows", "k_cols", "k_interp")[dom]
    rec = pmc.load_traffic(args.traffic_record, kname, N=N, B=B, L=info["L"], sigma=info["sigma"],
                           kernel_width=info["kernel_width"], ranks=[info["min_rank"], info["max_rank"]])
    traffic = rec["traffic_bytes"] if rec else None
    alg_bytes = by[dom] / lps[dom]
    if dom == 2:
        achieved = fl / lps[2] / (per_launch_ms[2] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP32_PEAK_TFLOPS, traffic=traffic, kernel=kname,
                    peak_nonpacked=FP32_NONPACKED_TFLOPS, frac_nonpacked=achieved / FP32_NONPACKED_TFLOPS,
                    flops_per_launch=fl / lps[2],
                    flops_formula="sum over wedges of N^2 q (4 w^2 + 4 w + 8) per right-hand side, true rank q")
    else:
        achieved = alg_bytes / (per_launch_ms[dom] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel=kname)
    roof.update(algorithmic_bytes=alg_bytes, ms_per_launch=per_launch_ms[dom],
                traffic_unit="HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                hbm_copy_gbs=copy_gbs)
    stages = {}
    for i, name in enumerate(STAGES):
        bpl = by[i] / max(1e-9, lps[i])
        gbs = bpl / (per_launch_ms[i] * 1e-3) / 1e9 if per_launch_ms[i] > 0 else None
        stages[name] = dict(ms_per_step=stage_ms[i], ms_per_launch=per_launch_ms[i], launches_per_step=lps[i],
                            algorithmic_bytes_per_launch=bpl, gbs=gbs,
                            hbm_frac=gbs / HBM_PEAK_GBS if gbs else None,
                            hbm_frac_of_copy=gbs / copy_gbs if gbs else None)
    stages["interp_combine"]["tflops"] = fl / (stage_ms[2] * 1e-3) / 1e12
    stages["interp_combine"]["fp32_frac"] = stages["interp_combine"]["tflops"] / FP32_PEAK_TFLOPS
    res = dict(metric="FIO applies/s at N=1024, rel-l2<=1e-4", value=value, unit="applies/s", n_gpus=1,
               steps=steps, warmup=args.warmup, ms_per_step=1e3 * elapsed / steps, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="c64 (fp32 data, fp64 phase and points)", data="synthetic",
               config=dict(workload="N=%d c1/c2 ellipse phase (scale 1), B=%d complex-Gaussian right-hand sides, "
                                    "tol %g, exact randomized-separation factors (%s), %s"
                                    % (N, B, args.tol, args.factor_mode if args.factor_mode != "auto" else "stored",
                                       "autotuned" if fixed is None else "fixed plan"),
                           N=N, batch=B, tol=args.tol, wedges=info["L"], ranks=[info["min_rank"], info["max_rank"]],
                           kernel_width=info["kernel_width"], sigma=info["sigma"],
                           sep_tol_frac=best["sep_tol_frac"], nufft_tol_frac=best["nufft_tol_frac"],
                           plan_s=plan_s, tuned=fixed is None, factor_bytes=info["factor_bytes"],
                           parallelism="single GPU"),
               roofline=roof, stages=stages,
               comparison=dict(per_rhs_loop_applies_per_s=single_value, batched_applies_per_s=value))
    # accuracy gate: every right-hand side against the FP64 oracle
    log("oracle check on %d sampled outputs x %d RHS" % (args.cpu_samples, B))
    xs, refv, dt, threads = oracle_check(N, 2, (1.0,), fh, args.cpu_samples, seed=4321)
    got = out.cpu().numpy().reshape(B, N * N)[:, xs].astype(np.complex128)
    errs = [float(np.linalg.norm(got[b] - refv[b]) / np.linalg.norm(refv[b])) for b in range(B)]
    res["rel_l2_vs_oracle"] = max(errs)
    res["rel_l2_vs_oracle_per_rhs"] = errs
    res["oracle_samples"] = int(args.cpu_samples)
    if args.no_cpu_baseline:
        res["cpu_baseline"] = None
    else:
        log("CPU oracle baseline: one thread on %d outputs" % args.cpu_one_thread_samples)
        res["cpu_baseline"] = cpu_baseline(N, 2, (1.0,), fh, args.cpu_samples, dt, threads,
                                           args.cpu_one_thread_samples)
    bad = max(errs) > args.tol
    if bad:
        res["invalid"] = "relative l2 error %.3e above the budget %.1e" % (max(errs), args.tol)
        res["value"] = None
    print(json.dumps(res), flush=True)
    if bad:
        sys.exit(3)


def run_batch512(args):
    """64 right-hand sides at N = 512 under the c1/c2 phase in one fused graph launch."""
    import numpy as np
    import torch

    import fio_inputs as fi
    from paper_math_0610051_amd import Plan, apply_multi

    N, B = 512, 64
    t0 = time.perf_counter()
    plan = Plan(N, "c1c2", args.tol, params=(1.0,), max_batch=B)
    plan_s = time.perf_counter() - t0
    rng = fi.rng_for(2, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    fd = torch.from_numpy(fh.astype(np.complex64)).cuda()
    out = torch.empty_like(fd)
    for _ in range(args.warmup):
        apply_multi([plan], [fd], [out])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        apply_multi([plan], [fd], [out])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    errs = [plan.probe_error(fd[b], out[b], nsamples=32) for b in range(0, B, 8)]
    info = plan.info()
    res = dict(metric="FIO applies/s, N=512, 64 right-hand sides in one graph launch", value=B * args.steps / el,
               unit="applies/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * el / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64 (fp32 data, fp64 phase)",
               data="synthetic",
               config=dict(workload="N=512 c1/c2 phase, B=64 complex-Gaussian right-hand sides, tol %g" % args.tol,
                           wedges=info["L"], ranks=[info["min_rank"], info["max_rank"]],
                           kernel_width=info["kernel_width"], plan_s=plan_s,
                           workspace_gb=info["workspace_bytes"] / 1e9),
               max_probe_rel_l2=max(errs), roofline=None, cpu_baseline=None)
    print(json.dumps(res), flush=True)


def run_uneven(args):
    import numpy as np
    import torch

    import fio_inputs as fi
    from paper_math_0610051_amd import Plan, apply_multi

    insts = fi.uneven_instances(32, seed=3000)
    plans, dev, fhs = [], [], []
    t0 = time.perf_counter()
    for inst in insts:
        kind, params = ("c1c2", (inst["scale"],)) if inst["family"] == "c1c2" else ("radial", (0.05, 0.5))
        plans.append(Plan(inst["N"], kind, args.tol, params=params))
        fh = fi.fhat_from_f(fi.instance_field(inst))
        fhs.append(fh)
        dev.append(torch.from_numpy(fh.astype(np.complex64)).cuda())
    plan_s = time.perf_counter() - t0
    outs = [torch.empty_like(d) for d in dev]
    for _ in range(args.warmup):
        apply_multi(plans, dev, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        apply_multi(plans, dev, outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # per-instance sequential applies for comparison
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        for p, d, o in zip(plans, dev, outs):
            p.apply(d, o)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    errs = []
    for p, d, o in zip(plans, dev, outs):
        errs.append(p.probe_error(d, o, nsamples=64))
    res = dict(metric="FIO applies/s, 32 uneven instances N in {128..1024}, one fused launch", value=32 * args.steps / el,
               unit="applies/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * el / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64 (fp32 data, fp64 phase)",
               data="synthetic",
               config=dict(workload="32 instances: N ~ U{128,256,512,1024}, c1/c2 (scale U[0.5,1.5]) or rho(x)|xi|, "
                                    "complex Gaussian or 20 Gaussian bumps, tol %g" % args.tol,
                           Ns=[i["N"] for i in insts], plan_s=plan_s),
               comparison=dict(sequential_applies_per_s=32 * max(1, args.steps // 2) / seq),
               max_instance_rel_l2_probe=max(errs), roofline=None, cpu_baseline=None)
    print(json.dumps(res), flush=True)


def run_learned(args):
    import numpy as np
    import torch

    import fio_inputs as fi
    from paper_math_0610051_amd import Learned, Plan

    N, B = args.N, args.batch
    net = Learned(N, "c1c2", (1.0,), seed=7)
    t0 = time.perf_counter()
    net.generate(fi.training_scales(64), x_samples=args.learned_samples, r_cols=48)
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = net.train(args.learned_steps, batch=args.learned_batch, lr=args.learned_lr, lr_final=1e-5)
    train_s = time.perf_counter() - t0
    held = fi.heldout_scales(16)
    net.generate(held, x_samples=1024, r_cols=48)
    held_loss = net.eval()
    rows = []
    rng = fi.rng_for(4, 1)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    fd = torch.from_numpy(fh.astype(np.complex64)).cuda()
    out = torch.empty_like(fd)
    for s in held[[2, 7, 13]]:
        for tol in (args.learned_tol, args.tol):
            t0 = time.perf_counter()
            pe = Plan(N, "c1c2", tol, params=(float(s),), max_batch=B, factor_mode="stored")
            exact_s = time.perf_counter() - t0
            t0 = time.perf_counter()
            pl = Plan(N, "c1c2", tol, params=(float(s),), max_batch=B, learned=net, learned_scale=float(s))
            learned_s = time.perf_counter() - t0
            il, ie = pl.info(), pe.info()
            el = time_applies(pl, fd, out, max(2, args.steps // 4), 1)
            err_l = pl.probe_error(fd[0], out[0], nsamples=96)
            ee = time_applies(pe, fd, out, max(2, args.steps // 4), 1)
            err_e = pe.probe_error(fd[0], out[0], nsamples=96)
            n = max(2, args.steps // 4)
            rows.append(dict(scale=float(s), tol=tol, learned_used=int(il["factor_mode"] == 3 and not il["fallback"]),
                             fallback=il["fallback"], learned_plan_s=learned_s, exact_plan_s=exact_s,
                             learned_applies_per_s=B * n / el, exact_applies_per_s=B * n / ee,
                             learned_err=err_l, exact_err=err_e, learned_attempt_sep_err=il["learned_sep_error"],
                             learned_attempt_ms=il["learned_ms"], plan_max_sep_err=il["max_sep_error"],
                             learned_ranks=[il["min_rank"], il["max_rank"]], exact_ranks=[ie["min_rank"], ie["max_rank"]],
                             learned_factor_bytes=il["factor_bytes"], exact_compressed_bytes=ie["compressed_bytes"]))
            pl.close()
            pe.close()
    res = dict(metric="learned vs exact factors at N=1024 (held-out phase scales)", value=None, unit="applies/s",
               n_gpus=1, steps=args.steps, warmup=1, higher_is_better=True, dtype="bf16 network, c64 apply",
               data="synthetic", network=dict(params=Learned.param_count(), weights_bytes_bf16=2 * Learned.param_count(),
                                              generate_s=gen_s, train_s=train_s, train_steps=args.learned_steps,
                                              final_batch_loss=loss, heldout_loss=held_loss),
               rows=rows, roofline=None, cpu_baseline=None, vs_baseline=None)
    print(json.dumps(res), flush=True)


def run_adjoint(args):
    """The adjoint apply (Section 3.5) on the benchmark's plan: B = 8
    complex-Gaussian grids g at N = 1024 -> Fourier coefficients of L*g,
    timed like the forward, and checked per right-hand side against the FP64
    adjoint direct sum at sampled frequencies."""
    import numpy as np
    import torch

    import fio_inputs as fi
    from oracle import direct as od

    N, B = args.N, args.batch
    fixed = tuple(float(v) for v in args.plan_params.split(",")) if args.plan_params else (40, 2.0, 0.4, 0.15, 5)
    plan, plan_s, best = tuned_plan(N, args.tol, B, fixed, args.factor_mode)
    info = plan.info()
    rng = fi.rng_for(5, 0)
    g = fi.complex_gaussian(N, rng, B=B)
    gd = torch.from_numpy(g.astype(np.complex64)).cuda()
    out = torch.empty_like(gd)
    for _ in range(args.warmup):
        plan.apply_adjoint(gd, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply_adjoint(gd, out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # forward on the same plan, for comparison
    fwd = torch.empty_like(gd)
    plan.apply(gd, fwd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(gd, fwd)
    torch.cuda.synchronize()
    el_f = time.perf_counter() - t0
    od.build(force=False)
    ks = np.sort(np.random.default_rng(77).choice(N * N, size=args.adjoint_samples, replace=False))
    log("adjoint oracle check on %d frequencies x %d RHS" % (ks.size, B))
    refv = od.direct_adjoint(N, 2, (1.0,), g, ks)
    got = out.cpu().numpy().reshape(B, N * N)[:, ks].astype(np.complex128)
    errs = [float(np.linalg.norm(got[b] - refv[b]) / np.linalg.norm(refv[b])) for b in range(B)]
    res = dict(metric="FIO adjoint applies/s at N=%d, rel-l2<=%g" % (N, args.tol),
               value=B * args.steps / el, unit="applies/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * el / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="c64 (fp32 data, fp64 phase and points)", data="synthetic",
               config=dict(workload="adjoint L* of the N=%d c1/c2 plan (L=%d, sigma=%g, w=%d, ranks %d..%d), "
                                    "B=%d complex-Gaussian grids" % (N, info["L"], info["sigma"],
                                                                      info["kernel_width"], info["min_rank"],
                                                                      info["max_rank"], B),
                           plan_s=plan_s),
               forward_applies_per_s=B * args.steps / el_f, rel_l2_vs_oracle=max(errs),
               rel_l2_vs_oracle_per_rhs=errs, oracle_samples=int(ks.size), roofline=None, cpu_baseline=None)
    bad = max(errs) > args.tol
    if bad:
        res["invalid"] = "relative l2 error %.3e above the budget %.1e" % (max(errs), args.tol)
        res["value"] = None
    print(json.dumps(res), flush=True)
    if bad:
        sys.exit(3)


# The paper's Tables 3 and 4 (Matlab, one 2.6 GHz CPU): N -> (eps, preprocessing s, evaluation s, error, MB).
PAPER_TABLE3 = {64: (2.44e-3, 2.06, 3.89, 2.08e-3, 0.76), 128: (6.10e-4, 10.9, 24.5, 8.02e-4, 1.26),
                256: (1.53e-4, 81.0, 165.0, 1.00e-4, 2.01), 512: (3.81e-5, 467.0, 988.0, 4.22e-5, 3.06)}
PAPER_TABLE4 = {64: (2.44e-3, 21.8, 36.7, 7.30e-4, 0.37), 128: (6.10e-4, 109.0, 165.0, 4.00e-4, 0.59),
                256: (1.53e-4, 662.0, 846.0, 1.39e-4, 0.89), 512: (3.81e-5, 3420.0, 4430.0, 3.69e-5, 1.38)}


def run_paper(args):
    """The paper's own examples at eps = 10 N^-2: the ellipse phase of eq.
    (nrphase) (Table 3) and the circles of eq. (circlerad) with the Bessel
    amplitude of eq. (ellipses_amp) (Table 4), white-noise f, N = 64 ... 512;
    per row: plan and apply time, applies/s, ranks, factor storage and the
    relative l2 error against the FP64 direct sum at 512 sampled outputs (the
    paper used 100), beside the paper's own figures (context only)."""
    import numpy as np
    import torch

    import fio_inputs as fi
    from oracle import direct as od
    from paper_math_0610051_amd import Plan

    od.build(force=False)
    rows = []
    for table, kind, amp, paper in (("3", 4, 0, PAPER_TABLE3), ("4", 5, 1, PAPER_TABLE4)):
        for N in (64, 128, 256, 512):
            eps = 10.0 / N ** 2
            rng = fi.rng_for(6, N + amp)
            fh = fi.fhat_from_f(fi.white_noise_real(N, rng))
            fd = torch.from_numpy(fh.astype(np.complex64)).cuda()
            t0 = time.perf_counter()
            plan = Plan(N, kind, eps, params=(1.0,), amplitude="bessel" if amp else "one")
            plan_s = time.perf_counter() - t0
            out = torch.empty_like(fd)
            el = time_applies(plan, fd, out, args.steps, args.warmup)
            xs = fi.sample_points(N, 512, rng)
            got = out.cpu().numpy().astype(np.complex128).ravel()[xs]
            exact = od.direct(N, kind, (1.0,), fh, xs, amp=amp)
            err = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
            info = plan.info()
            pe = paper[N]
            rows.append(dict(table=table, N=N, eps=eps, rel_l2=err, meets_eps=err <= eps, plan_s=plan_s,
                             apply_s=el / args.steps, applies_per_s=args.steps / el, L=info["L"],
                             ranks=[info["min_rank"], info["max_rank"]], kernel_width=info["kernel_width"],
                             factor_mb=info["factor_bytes"] / 1e6, compressed_mb=info["compressed_bytes"] / 1e6,
                             paper=dict(eps=pe[0], preprocessing_s=pe[1], evaluation_s=pe[2], error=pe[3],
                                        storage_mb=pe[4])))
            log("table %s N=%d: err %.2e (eps %.2e), apply %.3f ms, ranks %d..%d"
                % (table, N, err, eps, 1e3 * el / args.steps, info["min_rank"], info["max_rank"]))
            plan.close()
    res = dict(metric="the paper's Table 3 / Table 4 examples at eps = 10 N^-2 (applies/s and error per N)",
               value=None, unit="applies/s", n_gpus=1, steps=args.steps, warmup=args.warmup, higher_is_better=True,
               dtype="c64 (fp32 data, fp64 phase, points and amplitude)", data="synthetic white noise",
               config=dict(workload="paper examples: ellipse phase (Table 3), circles with Bessel amplitude "
                                    "(Table 4), N = 64 ... 512"),
               rows=rows, roofline=None, cpu_baseline=None, vs_baseline=None)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("batched", "batch512", "uneven", "learned", "paper", "adjoint"),
                    default="batched")
    ap.add_argument("--adjoint-samples", type=int, default=2048)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--cpu-samples", type=int, default=3072)
    ap.add_argument("--cpu-one-thread-samples", type=int, default=160)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the per-RHS loop comparison")
    ap.add_argument("--factor-mode", choices=("auto", "stored", "regen"), default="auto",
                    help="batched workload: stored spatial factors or regenerated ones")
    ap.add_argument("--plan-params", default="", help="L,sigma,sep_tol_frac,nufft_tol_frac[,kernel_width] instead of autotuning")
    ap.add_argument("--traffic-record", default=os.path.join(ROOT, "profiles", "k_interp_traffic_N1024_B8_c1c2.json"))
    ap.add_argument("--learned-steps", type=int, default=150000)
    ap.add_argument("--learned-samples", type=int, default=4096)
    ap.add_argument("--learned-tol", type=float, default=1e-2)
    ap.add_argument("--learned-batch", type=int, default=8192)
    ap.add_argument("--learned-lr", type=float, default=2e-3)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the apply would shard by wedge, "
              "with one sum of the partial outputs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    {"batched": run_batched, "batch512": run_batch512, "uneven": run_uneven,
     "learned": run_learned, "paper": run_paper, "adjoint": run_adjoint}[args.workload](args)


if __name__ == "__main__":
    main()
