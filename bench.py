"""Benchmark of the batched FIO apply on one MI355X.

One step = one fio_apply_batch of B right-hand sides through the whole hot
path (window + row FFT, column FFT, interpolate + combine) at N = 1024 under
the c1/c2 ellipse phase, FP32 data with FP64 phase, tolerance 1e-4
relative l2.  Inputs are seeded complex Gaussian fields already resident in
device memory.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 1024] [--batch 8]
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 lanes x FMA (2 flop) x 2.4 GHz, non-packed FP32
STAGES = ("window_rowfft", "colfft", "interp_combine")


def stage_work(plan, B):
    """Algorithmic bytes and flops per stage for one apply of B right-hand sides.

    Per wedge (box B1 x B2, grid n1 x n2, rank q, |W| members), complex64 = 8 B:
      stage 0 reads fhat on W and gamma^xi (q per member), writes B1 * n2 * q;
      stage 1 reads B1 * n2 * q, writes n1 * n2 * q;
      stage 2 reads n1 * n2 * q and gamma^x (N^2 q, once per launch of up to
              4 right-hand sides), writes N^2 per right-hand side; its flops
              are N^2 (4 w^2 q + 8 q + 8) per wedge and right-hand side.
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
        q = wi["rank"] + (wi["rank"] & 1)
        if wi["rank"] == 0:
            continue
        B1, B2 = wi["box"]
        n1, n2 = wi["fine"]
        nm = wi["members"]
        by[0] += es * (nm + nm * q + B1 * n2 * q) * B
        by[1] += es * (B1 * n2 * q + n1 * n2 * q) * B
        by[2] += es * (n1 * n2 * q) * B
        gx_bytes += es * NN * q
        fl += NN * (4.0 * w * w * q + 8.0 * q + 8.0) * B
    launches2 = math.ceil(B / 4)
    by[2] += gx_bytes * launches2 + es * NN * B
    return by, fl


def cpu_baseline(N, phase_kind, params, fh, samples, seed):
    """Time the FP64 direct-sum oracle on a bounded sample of outputs (all host threads)."""
    import numpy as np
    from oracle import direct as od

    od.build(force=False)
    rng = np.random.default_rng(seed)
    xs = np.sort(rng.choice(N * N, size=samples, replace=False))
    t0 = time.perf_counter()
    ref = od.direct(N, phase_kind, params, fh, xs)
    dt = time.perf_counter() - t0
    B = fh.shape[0]
    # one full apply of B right-hand sides evaluates N^2 outputs; the sample evaluated `samples`
    full_s = dt * (N * N) / samples
    return dict(value=B / full_s, unit="applies/s", cores=od.max_threads(), kind="oracle",
                sample="%d random outputs x %d RHS of the N=%d c1/c2 workload (%.2e kernel terms) in %.1f s; "
                       "extrapolated to all N^2 outputs" % (samples, B, N, float(samples) * N * N, dt),
                seconds=dt), xs, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--cpu-samples", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the wedge sharding is "
              "described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fio_inputs as fi
    from paper_math_0610051_amd import Plan

    N, B = args.N, args.batch
    print("bench: N=%d B=%d tol=%g building plan" % (N, B, args.tol), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan = Plan(N, "c1c2", args.tol, params=(1.0,), max_batch=B)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    rng = fi.rng_for(4, 0)
    fh = fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B))
    fd = torch.from_numpy(fh.astype(np.complex64)).cuda()
    out = torch.empty_like(fd)
    print("bench: plan %.1f s, L=%d ranks %d..%d w=%d; warmup" % (plan_s, info["L"], info["min_rank"],
                                                               info["max_rank"], info["kernel_width"]),
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.apply(fd, out)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(fd, out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, launches = plan.profile_read()
    plan.profile(False)
    value = B * args.steps / elapsed
    by, fl = stage_work(plan, B)
    per_launch_ms = [ms[i] / max(1, launches[i]) for i in range(3)]
    stage_ms_per_step = [ms[i] / args.steps for i in range(3)]
    dom = int(np.argmax(stage_ms_per_step))
    launches_per_step = [launches[i] / args.steps for i in range(3)]
    if dom == 2:
        flops_per_launch = fl / launches_per_step[2]
        achieved = flops_per_launch / (per_launch_ms[2] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP32_VALU_PEAK_TFLOPS, traffic=None, kernel="k_interp")
    else:
        bytes_per_launch = by[dom] / launches_per_step[dom]
        achieved = bytes_per_launch / (per_launch_ms[dom] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=None, kernel=("k_rows", "k_cols")[dom])
    stages = {}
    for i, name in enumerate(STAGES):
        bpl = by[i] / max(1e-9, launches_per_step[i])
        stages[name] = dict(ms_per_step=stage_ms_per_step[i], ms_per_launch=per_launch_ms[i],
                            gbs=bpl / (per_launch_ms[i] * 1e-3) / 1e9 if per_launch_ms[i] > 0 else None,
                            launches_per_step=launches_per_step[i])
    stages["interp_combine"]["tflops"] = fl / args.steps * 0 + fl / (stage_ms_per_step[2] * 1e-3) / 1e12
    # accuracy and CPU baseline on the same sample
    res = dict(metric="FIO applies/s at N=1024, rel-l2<=1e-4", value=value, unit="applies/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * elapsed / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="c64 (fp32; fp64 phase)",
               data="synthetic",
               config=dict(workload="N=%d c1/c2 ellipse phase, B=%d complex-Gaussian RHS, tol %g, exact "
                                    "(stored) randomized-separation factors" % (N, B, args.tol),
                           N=N, batch=B, tol=args.tol, wedges=info["L"], ranks=[info["min_rank"], info["max_rank"]],
                           kernel_width=info["kernel_width"], plan_s=plan_s, parallelism="single GPU"),
               roofline=roof, stages=stages)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline on %d sampled outputs" % args.cpu_samples, file=sys.stderr, flush=True)
        cb, xs, refv = cpu_baseline(N, 2, (1.0,), fh, args.cpu_samples, seed=4321)
        got = out.cpu().numpy().reshape(B, N * N)[:, xs].astype(np.complex128)
        res["rel_l2_vs_oracle"] = float(np.linalg.norm(got - refv) / np.linalg.norm(refv))
        cb.pop("seconds")
        res["cpu_baseline"] = cb
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
