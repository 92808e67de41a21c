#!/usr/bin/env python
"""Throughput of the RGP distortion-correction hot path on one MI355X.

One step = one whole correction of one synthetic 3T-brain-shaped pair, 144x168x111, phase
encoding along dim 1, FP32: image pyramid (3 levels), OT initialisation on the coarsest level,
10 Gauss-Newton steps per level with 20 PCG iterations each (rtol 0) and Armijo line search,
prolongation between levels, and the Jacobian-modulation correction - all through rgp_correct.
Inputs are resident in HBM before the timed region.  The per-kernel lines time back-to-back
launches of each hot kernel at the finest level with HIP events on the stream they run on.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "volume pairs corrected/s at 144×168×111; loss_grad+gn_hvp HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pcg_step_c2_traffic.json")
KERNEL_SOURCES = ("paper_2403_10706_amd/csrc/pcg.hip", "paper_2403_10706_amd/csrc/rgp_internal.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the PCG step from committed rocprofv3 counters, if still valid."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def event_time_ms(fn, stream, reps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def cpu_baseline(pair, levels, gn_iters, pcg_iters):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload.

    Sample: the pyramid, OT on the coarsest level, ONE Gauss-Newton step (with the full PCG
    iteration count) on every level, the prolongations and the final correction.  The per-pair
    time is extrapolated by counting each level's measured GN step gn_iters times.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import rgp as orc

    Ip = pair.I_plus.astype(np.float32).astype(np.float64)
    Im = pair.I_minus.astype(np.float32).astype(np.float64)
    pe = pair.pe
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pyr = orc.pyramid(Ip, Im, pair.h, levels)
        P, M, hh = pyr[-1]
        b = orc.ot_init(P, M, pe, hh).b0
        t_fixed = time.perf_counter() - t0
        t_gn = 0.0
        for li in range(levels - 1, -1, -1):
            P, M, hh = pyr[li]
            if li < levels - 1:
                t1 = time.perf_counter()
                b = orc.prolong_field(b, P.shape, pe)
                t_fixed += time.perf_counter() - t1
            t1 = time.perf_counter()
            b, _ = orc.gauss_newton(P, M, b, pe, hh, gn_iters=1, pcg_iters=pcg_iters, pcg_rtol=0.0)
            t_gn += time.perf_counter() - t1
        t1 = time.perf_counter()
        orc.transform(Ip, b, pe, pair.h, 1.0)
        orc.transform(Im, b, pe, pair.h, -1.0)
        t_fixed += time.perf_counter() - t1
    sample_s = t_fixed + t_gn
    per_pair = t_fixed + gn_iters * t_gn
    return dict(value=1.0 / per_pair, unit="pairs/s", cores=1, kind="oracle",
                sample=(f"pyramid + OT + 1 of {gn_iters} GN steps (PCG {pcg_iters}) per level + "
                        f"prolongations + correction, {sample_s:.1f} s measured; per-pair time "
                        f"{per_pair:.1f} s extrapolated (GN step x {gn_iters}); FP64 NumPy, "
                        "1 thread"))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "per-pair work is independent, so pairs shard across GPUs with no communication.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2403_10706_amd import rgp

    rgp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    levels, gn_iters, pcg_iters = 3, 10, 20
    log("bench: generating the 144x168x111 pair (seed 1)")
    pair = synth.make_workload("c2")
    shape, pe = pair.shape, pair.pe
    dt = torch.float32
    Ip = torch.as_tensor(pair.I_plus).to(dev, dt).contiguous()
    Im = torch.as_tensor(pair.I_minus).to(dev, dt).contiguous()
    opts = rgp.Options(levels=levels, gn_iters=gn_iters, pcg_iters=pcg_iters, pcg_rtol=0.0)
    copts = opts.to_c()
    nbytes = rgp.workspace_size(rgp.OP_CORRECT, shape, pe, (1.0, 1.0, 1.0), dt, copts)
    ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(rgp.field_shape(shape, pe), dtype=dt, device=dev)
    Tp = torch.empty_like(Ip)
    Tm = torch.empty_like(Im)

    # The whole correction is captured once into a HIP graph (rgp_correct_plan) on a side
    # stream of default priority; one step = one replay.  The eager path is timed too.
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    torch.cuda.set_stream(side)   # every library call below is enqueued on `side`
    stream = side
    plan = rgp.Plan(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)

    def step():
        plan.launch(side)

    def timed(fn, steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(side)
        for _ in range(steps):
            fn()
        e1.record(side)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
        rgp.correct_into(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps (graph replay)")
    wall, gpu_ms = timed(step, args.steps)
    eager_wall, _ = timed(lambda: rgp.correct_into(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side),
                          max(3, args.steps // 4))
    eager_ms = 1e3 * eager_wall / max(3, args.steps // 4)
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps / wall
    log(f"bench: {ms_per_step:.3f} ms/pair wall (graph), {gpu_ms / args.steps:.3f} ms/pair on "
        f"the stream, eager {eager_ms:.3f} ms/pair")

    # ---- per-kernel rooflines at the finest level (algorithmic bytes / event-timed launch) ----
    N = int(np.prod(shape))
    Nb = int(np.prod(rgp.field_shape(shape, pe)))
    f = 4
    reps = args.kernel_reps
    jdsp, g, hd, ho = rgp.loss_grad(Ip, Im, b, pe)
    lg_ws = torch.zeros(rgp.workspace_size(rgp.OP_LOSS_GRAD, shape, pe, (1, 1, 1), dt), dtype=torch.uint8, device=dev)
    t_lg = event_time_ms(lambda: rgp.loss_grad_into(Ip, Im, b, pe, None, g, hd, ho, lg_ws),
                         stream, reps) / reps
    v = torch.randn_like(b)
    Hv = torch.empty_like(b)
    vhv = torch.empty(1, dtype=torch.float64, device=dev)
    t_hv = event_time_ms(lambda: rgp.gn_hvp_into(hd, ho, v, Hv, vhv, shape, pe, lg_ws),
                         stream, reps) / reps
    pcg_ws = torch.zeros(rgp.workspace_size(rgp.OP_PCG_SOLVE, shape, pe, (1, 1, 1), dt), dtype=torch.uint8, device=dev)
    x = torch.empty_like(b)
    rhs = -g
    m1, m2 = 20, 20 + reps
    t_p1 = event_time_ms(lambda: rgp.pcg_solve_into(hd, ho, rhs, x, shape, pe, m1, pcg_ws),
                         stream, 5) / 5
    t_p2 = event_time_ms(lambda: rgp.pcg_solve_into(hd, ho, rhs, x, shape, pe, m2, pcg_ws),
                         stream, 5) / 5
    t_pcg = (t_p2 - t_p1) / (m2 - m1)
    b0 = torch.empty_like(b)
    ot_ws = torch.zeros(rgp.workspace_size(rgp.OP_OT_INIT, shape, pe, (1, 1, 1), dt), dtype=torch.uint8, device=dev)
    t_ot = event_time_ms(lambda: rgp.ot_init_into(Ip, Im, pe, b0, ot_ws), stream, reps) / reps

    kernels = {}

    def add(name, bytes_per_launch, ms, note):
        gbps = bytes_per_launch / (ms * 1e-3) / 1e9
        kernels[name] = dict(bytes_per_launch=bytes_per_launch, us_per_launch=round(ms * 1e3, 3),
                             achieved_GBps=round(gbps, 1), frac=round(gbps / HBM_PEAK_GBPS, 4),
                             bytes_rule=note)
        log(f"bench: {name:10s} {ms * 1e3:8.2f} us  {gbps:8.1f} GB/s  ({gbps / HBM_PEAK_GBPS:.3f} of peak)")

    add("pcg_step", 10 * Nb * f, t_pcg, "reads x,r,p,w,diag,off; writes x,r,p,w (40 B/node)")
    add("loss_grad", 2 * N * f + 4 * Nb * f, t_lg, "reads I+,I-,b; writes grad,diag,off")
    add("gn_hvp", 4 * Nb * f, t_hv, "reads v,diag,off; writes Hv (16 B/node)")
    add("ot_init", 2 * N * f + Nb * f, t_ot, "reads I+,I- once; writes b0 (shift pass included in time)")

    dom = kernels["pcg_step"]
    traffic = measured_traffic()
    roofline = dict(bound="hbm", achieved=dom["achieved_GBps"], peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=dom["frac"], traffic=traffic, kernel="k_pcg_step<float,8>",
                    bytes_per_launch=dom["bytes_per_launch"], us_per_launch=dom["us_per_launch"])

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a bounded sample (about 10 s)")
        cpu = cpu_baseline(pair, levels, gn_iters, pcg_iters)
        log(f"bench: oracle {1.0 / cpu['value']:.1f} s/pair extrapolated")

    line = dict(
        metric=METRIC, value=round(value, 3), unit="pairs/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="3T-brain-shaped pair 144x168x111, PE dim 1, FP32 images and field, "
                    "3 levels x 10 GN x 20 PCG (rtol 0), OT init, Armijo",
                    shape=list(shape), pe_dim=pe, levels=levels, gn_iters=gn_iters,
                    pcg_iters=pcg_iters, global_batch=1),
        gpu_ms_per_step=round(gpu_ms / args.steps, 4), eager_ms_per_step=round(eager_ms, 4),
        roofline=roofline, kernels=kernels, cpu_baseline=cpu,
        device=torch.cuda.get_device_name(0),
    )
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
