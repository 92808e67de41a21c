#!/usr/bin/env python
"""Throughput of the RGP distortion-correction hot path on one MI355X.

One step = one whole correction of one synthetic 3T-brain-shaped pair, 144x168x111, phase
encoding along dim 1, FP32: image pyramid (3 levels), OT initialisation on the coarsest level,
10 Gauss-Newton steps per level with 20 PCG iterations each (rtol 0) and Armijo line search,
prolongation between levels, and the Jacobian-modulation correction - all through the C ABI.
Inputs are resident in HBM before the timed region.  The correction is captured once into a HIP
graph (rgp_correct_plan) and one step is one replay; an eager pass of the same correction follows
with the library's kernel timing on (HIP events recorded at the start and end of every hot
kernel, rgp_timing_*), from which the per-kernel rooflines are computed.  The roofline's
`achieved` counts 52 B per cell per PCG iteration (the hot-path measurement table's figure);
`moved_bytes` beside it counts the 40 B per node the fused PCG kernel must move.

The same line carries the batched leg (`batch`, unless --batch-pairs 0): 32 uneven pairs
(BF16 images scaled x1000, FP32 field, same schedule) corrected by one batched graph against one
graph per pair, and the batched Gauss-Newton launches timed in an eager batched correction (their
working set is HBM-resident, ~2.8 GB per finest-level PCG iteration), and `cpu_baseline`: the
FP64 oracle's whole correction of the headline pair on one thread of the host.  `solvers` holds
the other per-level solvers on the headline pair and schedule (L-BFGS, ADMM: pairs/s of their own
captured plans) and the least-squares correction of the Gauss-Newton field (ms per call).

Prints ONE JSON line on stdout; progress goes to stderr.

Other modes (profiling helpers; their output goes under profiles/):
  --pmc-probe                 a plain 256 MiB elementwise copy, then one PCG solve on the finest
                              level (the workload for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)
  --traffic-summary F W       HBM traffic of the finest-level PCG step from the two --pmc runs
                              (directories F and W), scaled by the copy kernel's counters
  --profile-summary D         text summary of a rocprofv3 --kernel-trace --stats run in D
  --counter-summary D         per-kernel SQ instruction counters of a rocprofv3 --pmc run in D
  --batch N                   the batching benchmark: N uneven pairs, plain per-pair graphs
                              against one batched graph (its own JSON line)
  --batch-profile-summary D   per-kernel GB/s of the batched launches from a rocprofv3
                              --kernel-trace run of --batch 32 in D
  --range-summary D           per-level host and GPU time of the eager corrections from a
                              rocprofv3 --marker-trace --hip-runtime-trace --kernel-trace run in D
  --sweep                     pairs/s and the finest PCG step's GB/s for volumes from 64x64x48 to
                              320x320x256 (same schedule, FP32, PE dim 1)
"""
import argparse
import csv
import dataclasses
import glob
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "volume pairs corrected/s at 144×168×111; loss_grad+gn_hvp HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0
SHAPE, PE, LEVELS, GN_ITERS, PCG_ITERS = (144, 168, 111), 1, 3, 10, 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pcg_step_c2_traffic.json")
KERNEL_SOURCES = ("paper_2403_10706_amd/csrc/pcg.hip", "paper_2403_10706_amd/csrc/rgp_internal.hpp",
                  "paper_2403_10706_amd/csrc/rgp_launch.hpp")
COPY_MIB = 256
BATCH_LONG_MARCH = 16  # minimum PCG march of the second batched graph (option batch_march)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the finest-level PCG step from committed rocprofv3 counters, if
    they were taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


# ---------------------------------------------------------------------------------------------
# algorithmic bytes per launch (FP32 field f, image element size fi)

def algorithmic_bytes(rec, f=4, fi=4, maxit=PCG_ITERS):
    k, n, c, tag = rec["kernel"], rec["nodes"], rec["cells"], rec["tag"]
    if k == "pcg_step":
        if tag == 0:           # first iteration: reads rhs, diag, off; writes x, r, p, w
            return 7 * f * n
        if tag >= maxit:       # last update x += a p
            return 3 * f * n
        return 10 * f * n      # reads x, r, p, w, diag, off; writes x, r, p, w
    if k == "loss_grad":       # reads I+, I-, b (and q); writes grad, diag, off (and b + g q)
        return 2 * fi * c + (6 if tag else 4) * f * n
    if k == "trial":           # reads I+, I-, b, q
        return 2 * fi * c + 2 * f * n
    if k == "hvp":             # reads v, diag, off; writes Hv
        return 4 * f * n
    if k == "ot":              # reads I+, I-; writes b0
        return 2 * fi * c + f * n
    if k == "shift":           # reads I+, I-
        return 2 * fi * c
    if k == "blur":            # reads b, writes the blurred b
        return 2 * f * n
    if k == "block_pcg":       # reads diag, off, grad; writes d (every iteration in registers)
        return 4 * f * n
    if k == "lsq":             # reads I+, I-, b; writes the corrected image
        return 3 * fi * c + f * n
    return 0


def table_rule_bytes(rec, f=4, fi=4):
    """Algorithmic bytes per launch under the hot-path measurement table's per-unit figures
    (N cells, Nb field nodes): a PCG iteration (HVP and CG vector updates, ~13 array passes)
    52 N; loss_grad with the Jacobi diagonal 2 N s_img + 3 Nb f, without it 2 N s_img + 2 Nb f;
    gn_hvp (recomputing from the images) 2 N s_img + 3 Nb f; ot_init 2 N s_img + Nb f."""
    k, n, c = rec["kernel"], rec["nodes"], rec["cells"]
    if k == "pcg_step":
        return 52 * c * f // 4
    if k in ("loss_grad", "hvp"):
        return 2 * fi * c + 3 * f * n
    if k == "ot":
        return 2 * fi * c + f * n
    return algorithmic_bytes(rec, f, fi)


BYTES_RULE = {
    "pcg_step": "full iteration: reads x,r,p,w,diag,off, writes x,r,p,w (40 B/node)",
    "loss_grad": "reads I+,I-,b[,q], writes grad,diag,off[,b+gq] (8 B/cell + 16 or 24 B/node)",
    "trial": "reads I+,I-,b,q (8 B/cell + 8 B/node)",
    "hvp": "reads v,diag,off, writes Hv (16 B/node)",
    "ot": "reads I+,I-, writes b0 (8 B/cell + 4 B/node)",
    "shift": "reads I+,I- (8 B/cell)",
    "blur": "reads b, writes blurred b (8 B/node)",
    "block_pcg": "reads diag,off,grad, writes d (16 B/node); the iterations run in registers",
    "lsq": "reads I+,I-,b, writes the corrected image (12 B/cell + 4 B/node)",
}


def summarize_records(recs, maxit=PCG_ITERS):
    """Group timed launches by kernel and volume; the PCG step keeps full iterations only and
    trial passes keep first passes (later passes exit early once a step is accepted)."""
    groups = {}
    for r in recs:
        if r["kernel"] == "pcg_step" and not (1 <= r["tag"] < maxit):
            continue
        if r["kernel"] == "trial" and r["tag"] != 1:
            continue
        key = (r["kernel"], r["nodes"], r["tag"] if r["kernel"] == "loss_grad" else 0)
        groups.setdefault(key, []).append(r)
    out = {}
    for (k, nodes, tag), rs in sorted(groups.items(),
                                      key=lambda kv: (kv[0][0], -kv[0][1], kv[0][2])):
        ms = [r["ms"] for r in rs]
        mean = sum(ms) / len(ms)
        med = statistics.median(ms)
        b = algorithmic_bytes(rs[0], maxit=maxit)
        gbps = b / (mean * 1e-3) / 1e9 if mean > 0 else 0.0
        name = f"{k}@{nodes}n" + ("+step" if (k == "loss_grad" and tag) else "")
        out[name] = dict(kernel=k, cells=rs[0]["cells"], nodes=nodes, grid=rs[0]["grid"],
                         launches=len(rs), us_mean=round(mean * 1e3, 3),
                         us_median=round(med * 1e3, 3), bytes_per_launch=b,
                         achieved_GBps=round(gbps, 1), frac=round(gbps / HBM_PEAK_GBPS, 4),
                         bytes_rule=BYTES_RULE[k])
    return out


# ---------------------------------------------------------------------------------------------

def host_cpu():
    """CPU model and the logical CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(pair, levels, gn_iters, pcg_iters):
    """The FP64 oracle, as it stands, on the whole correction of the same pair: pyramid, OT on
    the coarsest level, every Gauss-Newton step of every level (PCG pcg_iters, rtol 0), the
    prolongations and the final correction, on one thread (about 25 s)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import rgp as orc

    Ip = pair.I_plus.astype(np.float32).astype(np.float64)
    Im = pair.I_minus.astype(np.float32).astype(np.float64)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orc.solve(Ip, Im, pair.pe, pair.h, levels=levels, gn_iters=gn_iters,
                  pcg_iters=pcg_iters, pcg_rtol=0.0)
        per_pair = time.perf_counter() - t0
    model, ncpu, avail = host_cpu()
    return dict(value=1.0 / per_pair, unit="pairs/s", cores=1, kind="oracle",
                sample=(f"one whole correction of the same pair ({levels} levels x {gn_iters} GN "
                        f"x {pcg_iters} PCG, OT, correction), {per_pair:.1f} s; FP64 NumPy, one "
                        "thread"),
                host_cpu=model, host_logical_cpus=ncpu, cpus_available=avail)


# ---------------------------------------------------------------------------------------------
# profiling helpers

def pmc_probe():
    """Workload of the rocprofv3 --pmc runs: a plain elementwise copy of known size (256 MiB read,
    256 MiB written), then one 20-iteration PCG solve on the finest level of the bench pair."""
    import torch

    import synth
    from paper_2403_10706_amd import rgp

    rgp.load()
    dev = torch.device("cuda:0")
    src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    pair = synth.make_workload("c2")
    Ip = torch.as_tensor(pair.I_plus).to(dev, torch.float32).contiguous()
    Im = torch.as_tensor(pair.I_minus).to(dev, torch.float32).contiguous()
    b = torch.zeros(rgp.field_shape(pair.shape, pair.pe), dtype=torch.float32, device=dev)
    _, g, hd, ho = rgp.loss_grad(Ip, Im, b, pair.pe)
    x, its, rel = rgp.pcg_solve(hd, ho, -g, pair.shape, pair.pe, maxit=PCG_ITERS, rtol=0.0)
    torch.cuda.synchronize()
    log(f"pmc probe: PCG {int(its.item())} iterations, relres {float(rel.item()):.3e}")


def _csv_rows(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise SystemExit(f"no {pattern} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _counter(rows, counter):
    """(kernel name, grid size, value) per dispatch for one counter, in dispatch order."""
    out = []
    for r in sorted(rows, key=lambda r: int(r.get("Dispatch_Id", 0))):
        if r.get("Counter_Name") != counter:
            continue
        out.append((r["Kernel_Name"], int(r.get("Grid_Size", 0)), float(r["Counter_Value"])))
    return out


def traffic_summary(fetch_dir, write_dir):
    nb = SHAPE[0] * (SHAPE[1] + 1) * SHAPE[2]
    vals = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter(_csv_rows(d, "*counter_collection.csv"), counter)
        # the copy: the elementwise kernels over the largest grid that are not fills
        ew = [(g, v) for name, g, v in rows if "elementwise" in name and "Fill" not in name]
        gmax = max((g for g, _ in ew), default=0)
        copy = [v for g, v in ew if g == gmax]
        pcg = [(g, v) for name, g, v in rows if "k_pcg_step" in name]
        if not copy or not pcg:
            raise SystemExit(f"{counter}: copy or PCG dispatches missing in {d}")
        # the solve's launches in order: iteration 0, full iterations, last update; keep the full
        # ones (all on the finest grid)
        full = [v for _, v in pcg[1:-1]]
        vals[counter] = dict(copy_kib=statistics.median(copy),
                             pcg_kib=statistics.median(full), pcg_launches=len(full))
    expect_kib = COPY_MIB * 1024.0
    sf = expect_kib / vals["FETCH_SIZE"]["copy_kib"]
    sw = expect_kib / vals["WRITE_SIZE"]["copy_kib"]
    fetch_b = vals["FETCH_SIZE"]["pcg_kib"] * sf * 1024.0
    write_b = vals["WRITE_SIZE"]["pcg_kib"] * sw * 1024.0
    algo = 40 * nb
    rec = dict(kernel="k_pcg_step",
               workload="144x168x111 PE dim 1 FP32, finest level, full PCG iteration",
               bytes_per_launch=int(round(fetch_b + write_b)), fetch_bytes=int(round(fetch_b)),
               write_bytes=int(round(write_b)), algorithmic_bytes=algo,
               traffic_over_algorithmic=round((fetch_b + write_b) / algo, 4),
               fetch_kib_raw=vals["FETCH_SIZE"]["pcg_kib"],
               write_kib_raw=vals["WRITE_SIZE"]["pcg_kib"],
               copy_fetch_kib_raw=vals["FETCH_SIZE"]["copy_kib"],
               copy_write_kib_raw=vals["WRITE_SIZE"]["copy_kib"],
               copy_expected_kib=expect_kib, scale_fetch=round(sf, 6), scale_write=round(sw, 6),
               launches=vals["FETCH_SIZE"]["pcg_launches"], source_sha256=kernel_source_hash(),
               commands=["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <F> -o run -- "
                         "python3 bench.py --pmc-probe",
                         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <W> -o run -- "
                         "python3 bench.py --pmc-probe",
                         "python3 bench.py --traffic-summary <F> <W>"])
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def counter_summary(d):
    """Per-kernel means of the SQ counters of a rocprofv3 --pmc run (one row per kernel name and
    grid): instructions per wavefront by kind, and the share of busy cycles."""
    rows = _csv_rows(d, "*counter_collection.csv")
    names = sorted({r["Counter_Name"] for r in rows})
    per = {}
    for r in rows:
        key = (r["Kernel_Name"].split("(")[0][:60], int(r.get("Grid_Size", 0)))
        per.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print(f"# rocprofv3 --pmc {' '.join(names)}: mean per dispatch; per-wave figures divide by SQ_WAVES")
    hdr = f"{'kernel':60s} {'grid':>9s} {'n':>5s} " + " ".join(f"{n[8:] if n.startswith('SQ_INSTS_') else n:>12s}" for n in names)
    print(hdr)
    for (k, g), c in sorted(per.items(), key=lambda kv: -kv[0][1]):
        n = len(next(iter(c.values())))
        means = {name: statistics.mean(v) for name, v in c.items()}
        waves = means.get("SQ_WAVES", 0.0)
        cols = []
        for name in names:
            v = means.get(name, float("nan"))
            if name.startswith("SQ_INSTS_") and waves > 0:
                v = v / waves   # per wavefront
            cols.append(f"{v:12.1f}")
        print(f"{k:60s} {g:9d} {n:5d} " + " ".join(cols))


def profile_summary(d):
    """Text summary of a rocprofv3 --kernel-trace --stats run: the per-kernel statistics table,
    then every kernel split by grid size (mean and median duration per launch)."""
    stats = _csv_rows(d, "*kernel_stats.csv")
    trace = _csv_rows(d, "*kernel_trace.csv")
    print("== rocprofv3 kernel statistics (per kernel name) ==")
    print(f"{'kernel':70s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r in stats[:30]:
        name = r["Name"][:70]
        print(f"{name:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    groups = {}
    for r in trace:
        name = r["Kernel_Name"].split("(")[0]
        key = (name, int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups.setdefault(key, []).append(dur)
    # PCG solves: runs of consecutive k_pcg_step launches on one grid (iteration 0, the full
    # iterations, the last update); the interior launches are the full iterations
    trace_sorted = sorted(trace, key=lambda r: int(r["Start_Timestamp"]))
    runs, cur, cur_grid = [], [], None
    for r in trace_sorted:
        name = r["Kernel_Name"]
        g = int(r["Grid_Size_X"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if "k_pcg_step" in name and (cur_grid is None or g == cur_grid):
            cur.append(dur)
            cur_grid = g
            continue
        if cur:
            runs.append((cur_grid, cur))
        cur, cur_grid = ([dur], g) if "k_pcg_step" in name else ([], None)
    if cur:
        runs.append((cur_grid, cur))
    interior = {}
    for g, v in runs:
        interior.setdefault(g, []).extend(v[1:-1])
    print()
    print("== k_pcg_step, full iterations only (interior launches of each solve) ==")
    print(f"{'grid_threads':>12s} {'n':>6s} {'mean_us':>9s} {'median_us':>9s}")
    for g, v in sorted(interior.items(), key=lambda kv: -kv[0]):
        if v:
            print(f"{g:12d} {len(v):6d} {sum(v) / len(v):9.2f} {statistics.median(v):9.2f}")
    print()
    print("== per kernel and grid (from the kernel trace) ==")
    print(f"{'kernel':62s} {'grid_threads':>12s} {'wg':>5s} {'n':>6s} {'mean_us':>9s} "
          f"{'median_us':>9s} {'total_ms':>9s}")
    for (name, gx, wg), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:40]:
        print(f"{name[-62:]:62s} {gx:12d} {wg:5d} {len(v):6d} {sum(v) / len(v):9.2f} "
              f"{statistics.median(v):9.2f} {sum(v) / 1e3:9.3f}")


def range_summary(d):
    """Per-level figures of the eager corrections in a rocprofv3 --marker-trace
    --hip-runtime-trace --kernel-trace run: the library's ROCTx ranges ("rgp: correction",
    "rgp: level L", "rgp: Gauss-Newton step k") give each launch its correction, level and step
    (through the launch call's correlation id).  Per Gauss-Newton step: the host time spent
    enqueueing it, the GPU span of its kernels (first start to last end) and their summed
    duration; corrections are grouped by their number of levels."""
    import bisect
    marks = _csv_rows(d, "*marker_api_trace.csv")
    api = _csv_rows(d, "*hip_api_trace.csv")
    kern = _csv_rows(d, "*kernel_trace.csv")
    ranges = [(r["Function"], int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
              for r in marks if r.get("Function", "").startswith("rgp:")]
    launch_t = {r["Correlation_Id"]: int(r["Start_Timestamp"]) for r in api}
    launches = sorted((launch_t[r["Correlation_Id"]], int(r["Start_Timestamp"]),
                       int(r["End_Timestamp"])) for r in kern if r["Correlation_Id"] in launch_t)
    times = [t for t, _, _ in launches]

    def inside(a, b):
        return launches[bisect.bisect_left(times, a):bisect.bisect_right(times, b)]

    def within(name, a, b):
        return [(m, x, y) for m, x, y in ranges if m.startswith(name) and a <= x and y <= b]

    table = {}
    for _, ca, cb in [r for r in ranges if r[0] == "rgp: correction"]:
        if not inside(ca, cb):
            continue   # recorded into a graph: nothing launched
        lvs = within("rgp: level ", ca, cb)
        nlev = len(lvs)
        for m, la, lb in lvs:
            for _, sa, sb in within("rgp: Gauss-Newton step", la, lb):
                ks = inside(sa, sb)
                if ks:
                    table.setdefault((nlev, int(m.split()[-1])), []).append((sb - sa, ks))
    print("== eager corrections by level (library ROCTx ranges; means per Gauss-Newton step) ==")
    print(f"{'levels':>6s} {'level':>5s} {'steps':>6s} {'kernels':>8s} {'host_enqueue_us':>16s} "
          f"{'gpu_span_us':>12s} {'gpu_busy_us':>12s}")
    for (nlev, lv), rows in sorted(table.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        n = len(rows)
        host = sum(h for h, _ in rows) / n / 1e3
        span = sum(max(e for _, _, e in ks) - min(s0 for _, s0, _ in ks) for _, ks in rows) / n / 1e3
        busy = sum(sum(e - s0 for _, s0, e in ks) for _, ks in rows) / n / 1e3
        nk = sum(len(ks) for _, ks in rows) / n
        print(f"{nlev:6d} {lv:5d} {n:6d} {nk:8.1f} {host:16.1f} {span:12.1f} {busy:12.1f}")


def copy_reference(dev, stream, reps=10):
    """Measured bandwidth of a plain device-to-device copy (torch's copy kernel) at two sizes:
    one that fits the 256 MB Infinity Cache together with its source (like the PCG step's working
    set at 144x168x111) and one well beyond it (HBM-resident).  Traffic = bytes read + written."""
    import torch
    out = []
    for mib in (64, 1024):
        n = mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        gbps = 2 * n * 4 / (us * 1e3)
        out.append(dict(traffic_MiB=2 * mib, us=round(us, 2), GBps=round(gbps, 1),
                        frac=round(gbps / HBM_PEAK_GBPS, 4)))
        del src, dst
    return out


def batch_level_bytes(n=32, levels=LEVELS, img_bytes=2, f=4):
    """Algorithmic bytes per batched launch on each pyramid level (finest first) of the uneven
    batch (BF16 images, FP32 field): the sums over the pairs of the per-volume rules."""
    import numpy as np

    from synth.phantom import batch_specs
    out = []
    shapes = [(tuple(sp["shape"]), sp["pe"]) for sp in batch_specs(n)]
    for lv in range(levels):
        N = Nb = 0
        for shape, pe in shapes:
            s = shape
            for _ in range(lv):
                s = tuple((x + 1) // 2 for x in s)
            N += int(np.prod(s))
            Nb += int(np.prod([x + (1 if d == pe else 0) for d, x in enumerate(s)]))
        out.append(dict(level=lv, cells=N, nodes=Nb,
                        pcg_step=10 * Nb * f,
                        loss_grad=2 * N * img_bytes + 6 * Nb * f,
                        trial=2 * N * img_bytes + 2 * Nb * f))
    return out


def batch_profile_summary(d):
    """Per-kernel GB/s of the batched launches (k_pcg_step_batch, k_loss_grad_batch and the
    single-candidate k_trial_batch) in a rocprofv3 --kernel-trace run of `bench.py --batch 32`.
    Each kernel's launches are grouped by grid size, largest grid = finest level; the median
    launch duration is set against the level's algorithmic bytes (full PCG iterations; loss_grad
    applying the step; the gamma = 1 trial pass)."""
    trace = _csv_rows(d, "*kernel_trace.csv")
    lv = batch_level_bytes()
    print("# batched launches of the uneven 32-pair batch (BF16 images, FP32 field, 3 levels x 10 GN x 20 PCG)")
    print("# bytes per launch: sums over the 32 pairs of 40 B/node (PCG step), 4 B/cell + 24 B/node")
    print("# (loss_grad applying the step), 4 B/cell + 8 B/node (trial, gamma = 1)")
    print(f"{'kernel':18s} {'level':>5s} {'grid':>9s} {'n':>5s} {'median_us':>10s} {'MB':>9s} "
          f"{'GB/s':>8s} {'frac':>6s}")
    rows = []
    for key, match in (("pcg_step", "k_pcg_step_batch"), ("loss_grad", "k_loss_grad_batch"),
                       ("trial", "k_trial_batch")):
        groups = {}
        for r in trace:
            name = r["Kernel_Name"]
            if match not in name:
                continue
            if key == "trial" and ", 1, 256>" not in name:
                continue  # the multi-candidate pass, a no-op once gamma = 1 is accepted
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups.setdefault(int(r["Grid_Size_X"]), []).append(dur)
        for level, (grid, v) in enumerate(sorted(groups.items(), key=lambda kv: -kv[0])[:LEVELS]):
            med = statistics.median(v)
            by = lv[level][key]
            gbps = by / (med * 1e3)
            rows.append(dict(kernel=key, level=level, grid=grid, n=len(v), us_median=round(med, 2),
                             bytes=by, GBps=round(gbps, 1), frac=round(gbps / HBM_PEAK_GBPS, 4)))
            print(f"{key:18s} {level:5d} {grid:9d} {len(v):5d} {med:10.2f} {by / 1e6:9.1f} "
                  f"{gbps:8.1f} {gbps / HBM_PEAK_GBPS:6.3f}")
    return rows


# ---------------------------------------------------------------------------------------------
# batching: the uneven batch of pairs, plain per-pair graphs against one batched graph

def _gen_batch_pair(args):
    i, n, scale = args
    import numpy as np

    import synth
    p = synth.make_batch_pair(i, n=n, scale=scale)
    return (p.I_plus.astype(np.float32), p.I_minus.astype(np.float32),
            np.asarray(p.b_true, np.float32), p.pe, tuple(p.shape))


def gen_batch(n, scale):
    """The uneven batch's pairs, generated in worker processes (call before the GPU is touched:
    the workers are forked)."""
    import multiprocessing as mp
    nproc = max(1, min(8, host_cpu()[2] // 2, n))
    with mp.get_context("fork").Pool(nproc) as pool:
        return pool.map(_gen_batch_pair, [(i, n, scale) for i in range(n)])


def batch_bench(pairs, steps, scale):
    """n synthetic pairs of uneven sizes (dims 96..200 x 96..200 x 60..132), PE along dim 0 or 1,
    BF16 images, FP32 field, 3 levels x 10 GN x 20 PCG.  Plain: one captured graph per pair
    (rgp_correct_plan) replayed pair after pair on one stream; batched: one captured graph for
    all pairs (rgp_correct_batch_plan).  Both use the same images; the final fields are compared
    with each other and with the true fields the pairs were synthesised from.  Then one eager
    batched correction (rgp_correct_batch) with kernel timing gives the batched launches'
    durations: their working set (level 0: ~2.8 GB per PCG iteration) is HBM-resident."""
    import numpy as np
    import torch

    from paper_2403_10706_amd import rgp

    rgp.load()
    n = len(pairs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bf = torch.bfloat16
    Ip = [torch.as_tensor(p[0]).to(dev, bf).contiguous() for p in pairs]
    Im = [torch.as_tensor(p[1]).to(dev, bf).contiguous() for p in pairs]
    pes = [p[3] for p in pairs]
    shapes = [p[4] for p in pairs]
    opts = rgp.Options(levels=LEVELS, gn_iters=GN_ITERS, pcg_iters=PCG_ITERS, pcg_rtol=0.0)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    torch.cuda.set_stream(side)
    # plain: one graph per pair, one shared workspace (the pairs run one after another)
    wsz = max(rgp.workspace_size(rgp.OP_CORRECT, sh, pe, (1.0, 1.0, 1.0), torch.float32,
                                 opts.to_c()) for sh, pe in zip(shapes, pes))
    ws = torch.zeros(wsz, dtype=torch.uint8, device=dev)
    bp_out = [torch.empty(rgp.field_shape(sh, pe), dtype=torch.float32, device=dev)
              for sh, pe in zip(shapes, pes)]
    Tp = [torch.empty_like(t) for t in Ip]
    Tm = [torch.empty_like(t) for t in Im]
    log(f"bench batch: autotuning {n} geometries")
    for i in range(n):
        rgp.autotune(shapes[i], pes[i], torch.float32, opts, ws=ws, stream=side)
    plans = [rgp.Plan(Ip[i], Im[i], pes[i], opts, bp_out[i], Tp[i], Tm[i], ws, stream=side)
             for i in range(n)]
    batch = rgp.BatchPlan(Ip, Im, pes, opts, stream=side)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    def plain():
        for pl in plans:
            pl.launch(side)

    plain()
    batch.launch(side)
    log(f"bench batch: timing {steps} plain passes and {steps} batched replays")
    t_plain = timed(plain, steps)
    t_batch = timed(lambda: batch.launch(side), steps)
    d_bp, e_plain, e_batch = [], [], []
    for i, p in enumerate(pairs):
        bb = batch.b[i].double().cpu().numpy()
        bq = bp_out[i].double().cpu().numpy()
        bt = p[2].astype(np.float64)
        d_bp.append(float(np.max(np.abs(bb - bq))))
        e_plain.append(float(np.sqrt(np.mean((bq - bt) ** 2))))
        e_batch.append(float(np.sqrt(np.mean((bb - bt) ** 2))))
    for pl in plans:
        pl.close()
    # one eager batched correction with kernel timing (the graph's launches are not timed)
    torch.cuda.synchronize()
    rgp.timing_start(1 << 16)
    batch.run_eager(side)
    torch.cuda.synchronize()
    recs = rgp.timing_stop(1 << 16)
    batch.close()
    # the same batch with the batched PCG launches marching at least BATCH_LONG_MARCH planes
    # per unit (option batch_march): fewer, longer units on the coarse levels
    opts_long = dataclasses.replace(opts, batch_march=BATCH_LONG_MARCH)
    batch_long = rgp.BatchPlan(Ip, Im, pes, opts_long, stream=side)
    batch_long.launch(side)
    t_long = timed(lambda: batch_long.launch(side), steps)
    d_lp = [float(torch.max(torch.abs(batch_long.b[i] - bp_out[i]))) for i in range(n)]
    batch_long.close()
    kernels = {}
    for name, rec in summarize_records(recs).items():
        if rec["kernel"] not in ("pcg_step", "loss_grad", "trial"):
            continue
        if rec["cells"] < sum(int(np.prod(sh)) for sh in shapes) // 80:
            continue   # a single pair's launch (the batch shares only the Gauss-Newton kernels)
        rb = dict(rec)
        # full PCG iterations, the gamma = 1 trial pass, loss_grad with or without the step
        tag = (1 if name.endswith("+step") else 0) if rec["kernel"] == "loss_grad" else 1
        b = algorithmic_bytes(dict(kernel=rec["kernel"], nodes=rec["nodes"], cells=rec["cells"],
                                   tag=tag), fi=2)
        rb["bytes_per_launch"] = b
        rb["achieved_GBps"] = round(b / (rec["us_mean"] * 1e3), 1)
        rb["frac"] = round(rb["achieved_GBps"] / HBM_PEAK_GBPS, 4)
        rb["bytes_rule"] = BYTES_RULE[rec["kernel"]].replace("8 B/cell", "4 B/cell (BF16)")
        kernels["batched:" + name] = rb
    for name, rec in kernels.items():
        log(f"bench batch: {name:40s} n={rec['launches']:4d} {rec['us_mean']:9.2f} us "
            f"{rec['achieved_GBps']:7.1f} GB/s frac {rec['frac']:.3f}")
    cells = int(sum(int(np.prod(sh)) for sh in shapes))
    out = dict(workload=f"{n} uneven pairs, dims 96-200 x 96-200 x 60-132, PE along dim 0 or 1, "
                        f"BF16 images x{scale:g}, FP32 field, {LEVELS} levels x {GN_ITERS} GN x "
                        f"{PCG_ITERS} PCG",
               unit="pairs/s", batched=round(n / t_batch, 3), plain=round(n / t_plain, 3),
               speedup=round(t_plain / t_batch, 3), ms_batched=round(1e3 * t_batch, 3),
               ms_plain=round(1e3 * t_plain, 3), steps=steps, cells=cells,
               max_abs_b_batched_vs_plain=max(d_bp),
               long_march=dict(batch_march=BATCH_LONG_MARCH, batched=round(n / t_long, 3),
                               ms_batched=round(1e3 * t_long, 3),
                               speedup=round(t_plain / t_long, 3),
                               max_abs_b_vs_plain=max(d_lp)),
               rms_error_vs_true_plain=round(float(np.mean(e_plain)), 6),
               rms_error_vs_true_batched=round(float(np.mean(e_batch)), 6),
               kernels=kernels)
    log(f"bench batch: plain {n / t_plain:.2f} pairs/s, batched {n / t_batch:.2f} pairs/s "
        f"(x{t_plain / t_batch:.2f}); max|b_batched - b_plain| = {max(d_bp):.2e}")
    log(f"bench batch: batch_march={BATCH_LONG_MARCH}: batched {n / t_long:.2f} pairs/s "
        f"(x{t_plain / t_long:.2f}); max|b - b_plain| = {max(d_lp):.2e}")
    return out


# ---------------------------------------------------------------------------------------------
# the other per-level solvers and the least-squares correction on the bench pair

def solver_legs(Ip, Im, pe, b_gn, side, steps):
    """L-BFGS (memory 10) and ADMM (PCG 20 per column) on the same pair and schedule (3 levels x
    10 iterations), each captured into its own plan and timed over `steps` replays (pairs/s,
    the status and the last level's final objective), and the least-squares correction (CGLS, at
    most 30 iterations, rtol 1e-6) of the Gauss-Newton field, timed over `steps` calls."""
    import torch

    from paper_2403_10706_amd import rgp
    shape = tuple(Ip.shape)
    dt = Ip.dtype
    out = dict(workload="the bench pair, 3 levels x 10 iterations of each solver (PCG 20, rtol 0)")
    for name, extra in (("lbfgs", dict(solver="lbfgs", lbfgs_memory=10)),
                        ("admm", dict(solver="admm"))):
        opts = rgp.Options(levels=LEVELS, gn_iters=GN_ITERS, pcg_iters=PCG_ITERS, pcg_rtol=0.0,
                           **extra)
        ws = torch.zeros(rgp.workspace_size(rgp.OP_CORRECT, shape, pe, (1.0, 1.0, 1.0), dt,
                                            opts.to_c()), dtype=torch.uint8, device=Ip.device)
        b = torch.empty(rgp.field_shape(shape, pe), dtype=dt, device=Ip.device)
        st = torch.empty(rgp.STAT_HEADER + LEVELS * GN_ITERS * rgp.STAT_FIELDS,
                         dtype=torch.float64, device=Ip.device)
        plan = rgp.Plan(Ip, Im, pe, opts, b, torch.empty_like(Ip), torch.empty_like(Im), ws,
                        stats=st, stream=side)
        plan.launch(side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.launch(side)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        plan.close()
        head, recs = rgp.parse_stats(st, LEVELS, GN_ITERS)
        out[name] = dict(pairs_per_s=round(1.0 / wall, 3), ms_per_pair=round(1e3 * wall, 3),
                         status=head["status"], J_last_step=recs[-1][-1]["J"])
        log(f"bench: {name}: {1.0 / wall:.2f} pairs/s ({1e3 * wall:.2f} ms), status "
            f"{head['status']}")
        # one eager correction with kernel timing: the solver's own kernels at the finest level
        rgp.timing_start(1 << 14)
        eager = rgp.correct(Ip, Im, pe, opts=opts, want_images=False, stream=side)
        side.synchronize()
        timed = rgp.timing_stop(1 << 14)
        _, erecs = rgp.parse_stats(eager["stats"], LEVELS, GN_ITERS)
        out[name]["kernels"] = leg_kernels(name, timed, erecs)
        for kname, kr in out[name]["kernels"].items():
            log(f"bench: {name} {kname}: {kr['achieved']} {kr['unit']} (frac {kr['frac']})")
        del ws, b, st, eager
    rgp.correct_lsq(Ip, Im, b_gn, pe, stream=side)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(side)
    for _ in range(steps):
        _, its = rgp.correct_lsq(Ip, Im, b_gn, pe, stream=side)
    e1.record(side)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out["lsq"] = dict(ms_per_call=round(ms, 3), cgls_iterations_max=int(its.max()))
    log(f"bench: least-squares correction {ms:.3f} ms (CGLS <= {int(its.max())} iterations)")
    rgp.timing_start(64)
    rgp.correct_lsq(Ip, Im, b_gn, pe, stream=side)
    side.synchronize()
    out["lsq"]["kernels"] = leg_kernels("lsq", rgp.timing_stop(64), None)
    return out


FP32_VECTOR_PEAK_TFLOPS = 157.3


def dht_flops(rec):
    """Flops of one Hartley pass by direct summation: every output of a line of length n is an
    n-term multiply-add sum (2 n flops), over every node of the field."""
    return 2 * (rec["tag"] >> 2) * rec["nodes"]


def _timed(recs, us, **kw):
    n = len(recs)
    return dict(launches=n, us_mean=round(us / max(n, 1), 3), **kw)


def leg_kernels(name, recs, levels_stats, f=4, fi=4):
    """The solver's own kernels at the finest level from one eager run with kernel timing:
    the Hartley passes (ALU: direct sums) and the block PCG of ADMM, the three direction launches
    of an L-BFGS step (bytes from the pairs each step used, read off the stats records), the
    least-squares kernel."""
    out = {}
    own = [r["nodes"] for r in recs if r["kernel"] in ("dht", "block_pcg", "lbfgs", "lsq")]
    if not own:
        return out
    top = max(own)
    fin = [r for r in recs if r["nodes"] == top]
    if name == "admm":
        dht = [r for r in fin if r["kernel"] == "dht"]
        if dht:
            us = 1e3 * sum(r["ms"] for r in dht)
            fl = sum(dht_flops(r) for r in dht)
            tf = fl / (us * 1e-6) / 1e12
            out["dht"] = _timed(dht, us, nodes=top, bound="alu", flops_per_launch=fl // len(dht),
                                achieved=round(tf, 2), peak=FP32_VECTOR_PEAK_TFLOPS,
                                unit="TFLOP/s", frac=round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
                                rule="2 n flops per node and pass (n-term sums along lines of "
                                     "length n); FP32 FMA, packed FP32 off")
        bp = [r for r in fin if r["kernel"] == "block_pcg"]
        if bp:
            us = 1e3 * sum(r["ms"] for r in bp)
            b = algorithmic_bytes(bp[0], f, fi)
            gbps = b * len(bp) / (us * 1e-6) / 1e9
            out["block_pcg"] = _timed(bp, us, nodes=top, bound="hbm", bytes_per_launch=b,
                                      achieved=round(gbps, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                                      frac=round(gbps / HBM_PEAK_GBPS, 4),
                                      rule=BYTES_RULE["block_pcg"],
                                      pcg_iters=bp[0]["tag"])
    elif name == "lbfgs":
        lb = [r for r in fin if r["kernel"] == "lbfgs"]
        st = levels_stats[-1] if levels_stats else []
        if lb and len(lb) == 3 * len(st) and all(math.isfinite(x["pcg_iters"]) for x in st):
            steps, us, byt, prev = [], 0.0, 0, 0
            for k, rec in enumerate(st):
                cnt = int(rec["pcg_iters"])
                dots = 4 * top if k == 0 else (20 + 8 * prev) * top
                comb = (8 + 8 * cnt) * top
                t = 1e3 * sum(r["ms"] for r in lb[3 * k:3 * k + 3])
                steps.append(dict(pairs=cnt, us=round(t, 3), bytes=dots + comb))
                us += t
                byt += dots + comb
                prev = cnt
            gbps = byt / (us * 1e-6) / 1e9
            out["direction"] = dict(
                nodes=top, steps=len(st), us_mean_per_step=round(us / len(st), 3), bound="hbm",
                bytes_per_step_mean=byt // len(st), achieved=round(gbps, 1), peak=HBM_PEAK_GBPS,
                unit="GB/s", frac=round(gbps / HBM_PEAK_GBPS, 4),
                rule="per step: pair and inner products (reads g, g_old, d and the window's s, y; "
                     "writes s, y: 20 + 8 p B/node), scalar recursion (one block), combination "
                     "(reads g and the kept s, y; writes d: 8 + 8 c B/node)",
                per_step=steps)
    elif name == "lsq":
        lq = [r for r in fin if r["kernel"] == "lsq"]
        if lq:
            us = 1e3 * sum(r["ms"] for r in lq)
            b = algorithmic_bytes(lq[0], f, fi)
            gbps = b * len(lq) / (us * 1e-6) / 1e9
            out["lsq"] = _timed(lq, us, nodes=top, cells=lq[0]["cells"], bound="hbm",
                                bytes_per_launch=b, achieved=round(gbps, 1), peak=HBM_PEAK_GBPS,
                                unit="GB/s", frac=round(gbps / HBM_PEAK_GBPS, 4),
                                rule=BYTES_RULE["lsq"])
    return out


def solver_cpu_baselines(pair, b_field, levels, iters, pcg_iters, sample=None):
    """The FP64 oracle on bounded samples of the solver legs, one thread: the whole correction
    with `sample[s]` of the `iters` iterations per level, and with none (pyramid, OT,
    prolongations and the correction alone), scaled linearly to `iters` iterations per level;
    the least-squares correction of the given field whole."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import lsq as olsq
    from oracle import rgp as orc

    sample = sample or dict(lbfgs=3, admm=2)
    Ip = pair.I_plus.astype(np.float32).astype(np.float64)
    Im = pair.I_minus.astype(np.float32).astype(np.float64)
    out = {}
    model, ncpu, avail = host_cpu()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orc.solve(Ip, Im, pair.pe, pair.h, levels=levels, gn_iters=0, pcg_iters=pcg_iters)
        fixed = time.perf_counter() - t0
        for name, extra in (("lbfgs", dict(solver="lbfgs", lbfgs_memory=10)),
                            ("admm", dict(solver="admm"))):
            k = sample[name]
            t0 = time.perf_counter()
            orc.solve(Ip, Im, pair.pe, pair.h, levels=levels, gn_iters=k, pcg_iters=pcg_iters,
                      pcg_rtol=0.0, **extra)
            tk = time.perf_counter() - t0
            per_pair = fixed + (tk - fixed) * iters / k
            out[name] = dict(value=1.0 / per_pair, unit="pairs/s", cores=1, kind="oracle",
                             sample=(f"{k} of {iters} iterations per level ({levels} levels, PCG "
                                     f"{pcg_iters}) {tk:.1f} s, without iterations {fixed:.1f} s; "
                                     f"per pair {per_pair:.1f} s scaled linearly in the "
                                     "iterations; FP64 NumPy, one thread"),
                             host_cpu=model)
        t0 = time.perf_counter()
        olsq.lsq_correct(Ip, Im, np.asarray(b_field, dtype=np.float64), pair.pe, pair.h)
        tl = time.perf_counter() - t0
        out["lsq"] = dict(value=round(1e3 * tl, 1), unit="ms per call", cores=1, kind="oracle",
                          sample="one whole least-squares correction (CGLS, at most 30 iterations, "
                                 f"rtol 1e-6) of the same field, {tl:.1f} s; FP64 NumPy, one thread",
                          host_cpu=model)
    return out


# ---------------------------------------------------------------------------------------------
# size sweep: the same schedule on volumes from 64x64x48 to 320x320x256

SWEEP_SHAPES = [(64, 64, 48), (96, 112, 74), (144, 168, 111), (200, 200, 132), (256, 256, 192),
                (320, 320, 256)]


def _sweep_images(shape, pe, dev, seed):
    """Smooth seeded stand-ins built on the device (the phantom generator is too slow on the
    host for the largest sizes): I- is I+ shifted by 3 cells along PE, scaled x1000."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    out = None
    for d, n in enumerate(shape):
        k = float(rng.integers(2, 5))
        ph = float(rng.uniform(0.0, 2.0 * np.pi))
        x = torch.arange(n, device=dev, dtype=torch.float32)
        f = 1.0 + 0.5 * torch.sin(2.0 * np.pi * k * x / n + ph)
        view = [1, 1, 1]
        view[d] = n
        f = f.view(view)
        out = f if out is None else out * f
    Ip = (1000.0 * out).contiguous()
    Im = torch.roll(Ip, shifts=3, dims=pe).contiguous()
    return Ip, Im


def size_sweep(steps):
    """Graph-replay throughput of the 3-level x 10 GN x 20 PCG correction (FP32, PE dim 1) per
    volume size, and the finest level's PCG step (median full iteration of one eager correction
    with kernel timing) against its 40 B/node."""
    import torch

    from paper_2403_10706_amd import rgp
    rgp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    torch.cuda.set_stream(side)
    dt, pe = torch.float32, 1
    opts = rgp.Options(levels=LEVELS, gn_iters=GN_ITERS, pcg_iters=PCG_ITERS, pcg_rtol=0.0)
    rows = []
    print(f"{'shape':>16s} {'field nodes':>12s} {'ms/pair':>9s} {'pairs/s':>9s} "
          f"{'PCG us':>8s} {'PCG GB/s':>9s} {'frac':>6s} {'march XL':>12s}")
    for i, shape in enumerate(SWEEP_SHAPES):
        Ip, Im = _sweep_images(shape, pe, dev, 50 + i)
        ws = torch.zeros(rgp.workspace_size(rgp.OP_CORRECT, shape, pe, (1.0, 1.0, 1.0), dt,
                                            opts.to_c()), dtype=torch.uint8, device=dev)
        b = torch.empty(rgp.field_shape(shape, pe), dtype=dt, device=dev)
        Tp, Tm = torch.empty_like(Ip), torch.empty_like(Im)
        xl = rgp.autotune(shape, pe, dt, opts, ws=ws, stream=side)
        plan = rgp.Plan(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)
        for _ in range(2):
            plan.launch(side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.launch(side)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        plan.close()
        rgp.timing_start(1 << 14)
        rgp.correct_into(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)
        torch.cuda.synchronize()
        recs = rgp.timing_stop(1 << 14)
        nb = max(r["nodes"] for r in recs if r["kernel"] == "pcg_step")
        full = [r["ms"] * 1e3 for r in recs if r["kernel"] == "pcg_step" and r["nodes"] == nb
                and 0 < r["tag"] < PCG_ITERS]
        us = statistics.median(full)
        gbps = 40.0 * nb / (us * 1e3)
        row = dict(shape=list(shape), nodes=int(nb), ms_per_pair=round(1e3 * wall, 3),
                   pairs_per_s=round(1.0 / wall, 2), pcg_us=round(us, 2),
                   pcg_GBps=round(gbps, 1), pcg_frac=round(gbps / HBM_PEAK_GBPS, 3),
                   march_xl=list(xl))
        rows.append(row)
        print(f"{'x'.join(map(str, shape)):>16s} {nb:12d} {1e3 * wall:9.3f} {1.0 / wall:9.2f} "
              f"{us:8.2f} {gbps:9.1f} {gbps / HBM_PEAK_GBPS:6.3f} {str(list(xl)):>12s}",
              flush=True)
        del Ip, Im, ws, b, Tp, Tm
        torch.cuda.empty_cache()
    print(json.dumps(dict(sweep=rows)))


# ---------------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eager-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--profile-summary", metavar="DIR")
    ap.add_argument("--counter-summary", metavar="DIR")
    ap.add_argument("--batch-profile-summary", metavar="DIR")
    ap.add_argument("--range-summary", metavar="DIR")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--batch", type=int, metavar="N", default=0,
                    help="the batching benchmark over N uneven pairs instead of the headline")
    ap.add_argument("--batch-scale", type=float, default=1000.0)
    ap.add_argument("--batch-pairs", type=int, default=32,
                    help="pairs of the batched leg of the default run (0: leave it out)")
    args = ap.parse_args()
    if args.traffic_summary:
        return traffic_summary(*args.traffic_summary)
    if args.profile_summary:
        return profile_summary(args.profile_summary)
    if args.range_summary:
        return range_summary(args.range_summary)
    if args.sweep:
        return size_sweep(max(3, min(args.steps, 10)))
    if args.counter_summary:
        return counter_summary(args.counter_summary)
    if args.batch_profile_summary:
        batch_profile_summary(args.batch_profile_summary)
        return None
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the "
              "per-pair work is independent, so pairs shard across GPUs with no communication.",
              file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        return pmc_probe()
    if args.batch:
        log(f"bench --batch: generating {args.batch} uneven pairs")
        res = batch_bench(gen_batch(args.batch, args.batch_scale), max(1, args.steps // 4),
                          args.batch_scale)
        print(json.dumps(res), flush=True)
        return None
    # the batched leg's pairs are generated first, in forked workers, before the GPU is touched
    batch_pairs = None
    if args.batch_pairs > 0:
        log(f"bench: generating the {args.batch_pairs} uneven pairs of the batched leg")
        batch_pairs = gen_batch(args.batch_pairs, args.batch_scale)

    import numpy as np
    import torch

    import synth
    from paper_2403_10706_amd import rgp

    rgp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("bench: generating the 144x168x111 pair (seed 1)")
    pair = synth.make_workload("c2")
    shape, pe = pair.shape, pair.pe
    assert tuple(shape) == SHAPE and pe == PE
    dt = torch.float32
    Ip = torch.as_tensor(pair.I_plus).to(dev, dt).contiguous()
    Im = torch.as_tensor(pair.I_minus).to(dev, dt).contiguous()
    opts = rgp.Options(levels=LEVELS, gn_iters=GN_ITERS, pcg_iters=PCG_ITERS, pcg_rtol=0.0)
    copts = opts.to_c()
    nbytes = rgp.workspace_size(rgp.OP_CORRECT, shape, pe, (1.0, 1.0, 1.0), dt, copts)
    ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(rgp.field_shape(shape, pe), dtype=dt, device=dev)
    Tp = torch.empty_like(Ip)
    Tm = torch.empty_like(Im)

    # The whole correction is captured once into a HIP graph (rgp_correct_plan) on a side
    # stream of default priority; one step = one replay.  The PCG march of every level is tuned
    # first (rgp_autotune, part of the setup like the capture).
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    torch.cuda.set_stream(side)   # every library call below is enqueued on `side`
    tuned_xl = rgp.autotune(shape, pe, dt, opts, ws=ws, stream=side)
    log(f"bench: tuned PCG march lengths per level (finest first): {tuned_xl}")
    plan = rgp.Plan(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)

    def eager():
        rgp.correct_into(Ip, Im, pe, opts, b, Tp, Tm, ws, stream=side)

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
        plan.launch(side)
        eager()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps (graph replay)")
    wall, gpu_ms = timed(lambda: plan.launch(side), args.steps)
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps / wall
    log(f"bench: {ms_per_step:.3f} ms/pair wall, {gpu_ms / args.steps:.3f} ms/pair on the stream")

    # ---- the same pair in the nonlinear regime: images x1000 (the distance term dominates, the
    # field reaches ~8 voxels and the line search backtracks); its own captured plan ----
    Ip_nl = Ip * 1000.0
    Im_nl = Im * 1000.0
    b_nl = torch.empty_like(b)
    st_nl = torch.empty(rgp.STAT_HEADER + LEVELS * GN_ITERS * rgp.STAT_FIELDS,
                        dtype=torch.float64, device=dev)
    plan_nl = rgp.Plan(Ip_nl, Im_nl, pe, opts, b_nl, torch.empty_like(Ip), torch.empty_like(Im),
                       ws, stats=st_nl, stream=side)
    for _ in range(max(1, args.warmup)):
        plan_nl.launch(side)
    wall_nl, _ = timed(lambda: plan_nl.launch(side), args.steps)
    _, recs_nl = rgp.parse_stats(st_nl, LEVELS, GN_ITERS)
    trials_nl = [int(r["trials"]) for lv in recs_nl for r in lv]
    plan_nl.close()
    nonlinear = dict(workload="the same pair with the images x1000 (same schedule)",
                     value=round(args.steps / wall_nl, 3), unit="pairs/s",
                     ms_per_step=round(1e3 * wall_nl / args.steps, 4),
                     armijo_trials_per_step=trials_nl,
                     steps_that_backtracked=sum(t > 1 for t in trials_nl),
                     max_abs_b=round(float(torch.max(torch.abs(b_nl))), 4))
    log(f"bench: nonlinear regime (x1000) {nonlinear['value']:.2f} pairs/s, "
        f"{nonlinear['steps_that_backtracked']} of {len(trials_nl)} steps backtracked")
    del Ip_nl, Im_nl

    # ---- the 7T-shaped pair: 200x200x132, PE dim 0, 4 levels, same schedule; its own plan ----
    pair3 = synth.make_workload("c3")
    opts3 = rgp.Options(levels=4, gn_iters=GN_ITERS, pcg_iters=PCG_ITERS, pcg_rtol=0.0)
    Ip3 = torch.as_tensor(pair3.I_plus).to(dev, dt).contiguous()
    Im3 = torch.as_tensor(pair3.I_minus).to(dev, dt).contiguous()
    ws3 = torch.zeros(rgp.workspace_size(rgp.OP_CORRECT, pair3.shape, pair3.pe, (1.0, 1.0, 1.0),
                                         dt, opts3.to_c()), dtype=torch.uint8, device=dev)
    b3 = torch.empty(rgp.field_shape(pair3.shape, pair3.pe), dtype=dt, device=dev)
    xl3 = rgp.autotune(pair3.shape, pair3.pe, dt, opts3, ws=ws3, stream=side)
    plan3 = rgp.Plan(Ip3, Im3, pair3.pe, opts3, b3, torch.empty_like(Ip3), torch.empty_like(Im3),
                     ws3, stream=side)
    for _ in range(max(1, args.warmup)):
        plan3.launch(side)
    wall3, _ = timed(lambda: plan3.launch(side), args.steps)
    plan3.close()
    # one eager correction with kernel timing: the finest level's kernels (5.3 M nodes)
    Tp3, Tm3 = torch.empty_like(Ip3), torch.empty_like(Im3)
    rgp.timing_start(1 << 14)
    timed(lambda: rgp.correct_into(Ip3, Im3, pair3.pe, opts3, b3, Tp3, Tm3, ws3, stream=side), 1)
    recs3 = rgp.timing_stop(1 << 14)
    nb3 = int(np.prod(rgp.field_shape(pair3.shape, pair3.pe)))
    k3 = {name: rec for name, rec in summarize_records(recs3).items() if rec["nodes"] == nb3}
    c3 = dict(workload="200x200x132 pair, PE dim 0, FP32, 4 levels x 10 GN x 20 PCG (7T-shaped)",
              value=round(args.steps / wall3, 3), unit="pairs/s",
              ms_per_step=round(1e3 * wall3 / args.steps, 4), tuned_march=list(xl3),
              max_abs_b=round(float(torch.max(torch.abs(b3))), 4), kernels=k3)
    log(f"bench: 200x200x132 pair {c3['value']:.2f} pairs/s ({c3['ms_per_step']:.3f} ms)")
    for name, rec in k3.items():
        log(f"bench: 200x200x132 {name:28s} n={rec['launches']:4d} {rec['us_mean']:8.2f} us  "
            f"{rec['achieved_GBps']:7.1f} GB/s  frac {rec['frac']:.3f}")
    del Ip3, Im3, ws3, b3, Tp3, Tm3

    # ---- eager pass with kernel timing: per-kernel durations from HIP events ----
    ne = max(1, args.eager_steps)
    rgp.timing_start(1 << 16)
    eager_wall, _ = timed(eager, ne)
    recs = rgp.timing_stop(1 << 16)
    eager_ms = 1e3 * eager_wall / ne
    log(f"bench: eager with kernel timing {eager_ms:.3f} ms/pair ({len(recs)} timed launches)")
    kernels = summarize_records(recs)

    # stand-alone calls at full resolution: loss_grad, gn_hvp, ot_init, the OT blur (R launches each)
    R = 20
    lg_ws = torch.zeros(rgp.workspace_size(rgp.OP_LOSS_GRAD, shape, pe, (1, 1, 1), dt),
                        dtype=torch.uint8, device=dev)
    ot_ws = torch.zeros(rgp.workspace_size(rgp.OP_OT_INIT, shape, pe, (1, 1, 1), dt),
                        dtype=torch.uint8, device=dev)
    g = torch.empty_like(b)
    hd = torch.empty_like(b)
    ho = torch.empty_like(b)
    v = torch.randn(b.shape, device=dev, dtype=dt)
    Hv = torch.empty_like(b)
    vhv = torch.empty(1, dtype=torch.float64, device=dev)
    b0 = torch.empty_like(b)
    bz = torch.zeros_like(b)
    torch.cuda.synchronize()
    rgp.timing_start(1 << 12)
    for _ in range(R):
        rgp.loss_grad_into(Ip, Im, bz, pe, None, g, hd, ho, lg_ws, stream=side)
    for _ in range(R):
        rgp.gn_hvp_into(hd, ho, v, Hv, vhv, shape, pe, lg_ws, stream=side)
    for _ in range(R):
        rgp.ot_init_into(Ip, Im, pe, b0, ot_ws, stream=side)
    b0b = torch.empty_like(b0)
    for _ in range(R):
        rgp.blur_field(b0, shape, pe, out=b0b, stream=side)
    torch.cuda.synchronize()
    solo = rgp.timing_stop(1 << 12)
    for name, rec in summarize_records(solo).items():
        kernels["standalone:" + name] = rec
    for name, rec in kernels.items():
        log(f"bench: {name:34s} n={rec['launches']:4d} {rec['us_mean']:8.2f} us "
            f"(median {rec['us_median']:7.2f})  {rec['achieved_GBps']:7.1f} GB/s  "
            f"frac {rec['frac']:.3f}")

    copy = copy_reference(dev, side)
    log("bench: plain copy " + ", ".join(f"{c['traffic_MiB']} MiB traffic {c['GBps']:.0f} GB/s"
                                         for c in copy))

    nb = int(np.prod(rgp.field_shape(shape, pe)))
    dom = next(r for r in kernels.values() if r["kernel"] == "pcg_step" and r["nodes"] == nb)
    traffic = measured_traffic()
    # achieved: the measurement table's per-unit figure for a PCG iteration (52 B per cell)
    # over the measured mean launch; moved_bytes: what this fused kernel must move (40 B/node)
    sb = table_rule_bytes(dict(kernel="pcg_step", nodes=dom["nodes"], cells=dom["cells"], tag=1))
    s_gbps = sb / (dom["us_mean"] * 1e3)
    roofline = dict(bound="hbm", achieved=round(s_gbps, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(s_gbps / HBM_PEAK_GBPS, 4), traffic=traffic,
                    kernel="k_pcg_step (finest level, 144x169x111 nodes, full PCG iterations)",
                    bytes_rule="52 B per cell per PCG iteration (HVP + CG vector updates)",
                    bytes_per_launch=sb, us_per_launch=dom["us_mean"],
                    us_median=dom["us_median"], launches=dom["launches"], grid=dom["grid"],
                    moved_bytes=dict(bytes_rule=dom["bytes_rule"],
                                     bytes_per_launch=dom["bytes_per_launch"],
                                     achieved=dom["achieved_GBps"], frac=dom["frac"]),
                    copy_reference=copy)

    solvers = solver_legs(Ip, Im, pe, b, side, max(2, args.steps // 4))
    b_host = b.double().cpu().numpy()
    solvers["gn"] = dict(pairs_per_s=round(value, 3), ms_per_pair=round(ms_per_step, 3))
    plan.close()
    batch = None
    if batch_pairs:
        batch = batch_bench(batch_pairs, max(1, args.steps // 4), args.batch_scale)
        del batch_pairs

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on one whole correction (about 25 s)")
        cpu = cpu_baseline(pair, LEVELS, GN_ITERS, PCG_ITERS)
        log(f"bench: oracle {1.0 / cpu['value']:.1f} s/pair ({cpu['host_cpu']})")
        log("bench: timing the FP64 oracle on samples of the solver legs (about 30 s)")
        for name, base in solver_cpu_baselines(pair, b_host, LEVELS, GN_ITERS, PCG_ITERS).items():
            solvers[name]["cpu_baseline"] = base
            log(f"bench: oracle {name}: {base['value']:.4g} {base['unit']}")

    line = dict(
        metric=METRIC, value=round(value, 3), unit="pairs/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="3T-brain-shaped pair 144x168x111, PE dim 1, FP32 images and field, "
                    "3 levels x 10 GN x 20 PCG (rtol 0), OT init, Armijo",
                    shape=list(shape), pe_dim=pe, levels=LEVELS, gn_iters=GN_ITERS,
                    pcg_iters=PCG_ITERS, global_batch=1, pcg_march_lengths=tuned_xl),
        gpu_ms_per_step=round(gpu_ms / args.steps, 4), eager_ms_per_step=round(eager_ms, 4),
        roofline=roofline, kernels=kernels, nonlinear=nonlinear, c3=c3, solvers=solvers,
        batch=batch,
        cpu_baseline=cpu,
        device=torch.cuda.get_device_name(0),
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
