"""Host logic of bench.py (no GPU): byte rules, record grouping, counter scaling and the
rocprofv3 trace summaries, on synthetic inputs."""
import csv
import io
import json
import os
import subprocess
import sys
from contextlib import redirect_stdout

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N_C2 = 144 * 168 * 111
NB_C2 = 144 * 169 * 111


def _rec(kernel, tag, ms=0.02, nodes=NB_C2, cells=N_C2, grid=448):
    return dict(kernel=kernel, tag=tag, ms=ms, nodes=nodes, cells=cells, grid=grid)


def test_gpus_above_one_exit_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_bytes_per_kernel_at_the_bench_shape():
    ab = bench.algorithmic_bytes
    assert ab(_rec("pcg_step", 5)) == 40 * NB_C2 == 108_051_840
    assert ab(_rec("pcg_step", 0)) == 28 * NB_C2          # iteration 0: rhs, diag, off in
    assert ab(_rec("pcg_step", 20)) == 12 * NB_C2         # last update x += a p
    assert ab(_rec("loss_grad", 0)) == 8 * N_C2 + 16 * NB_C2 == 64_703_232
    assert ab(_rec("loss_grad", 1)) == 8 * N_C2 + 24 * NB_C2 == 86_313_600
    assert ab(_rec("trial", 1)) == 8 * N_C2 + 8 * NB_C2 == 43_092_864
    assert ab(_rec("hvp", 0)) == 16 * NB_C2
    assert ab(_rec("ot", 0)) == 8 * N_C2 + 4 * NB_C2 == 32_287_680
    assert ab(_rec("shift", 0)) == 8 * N_C2
    assert ab(_rec("ot", 0), fi=2) == 4 * N_C2 + 4 * NB_C2  # BF16 images


def test_summarize_records_keeps_full_iterations_and_first_trial_passes():
    recs = [_rec("pcg_step", t, ms=0.5 if t in (0, 20) else 0.02) for t in range(21)]
    recs += [_rec("trial", 1, ms=0.015), _rec("trial", 2, ms=0.004)]
    recs += [_rec("loss_grad", 0, ms=0.018), _rec("loss_grad", 1, ms=0.022),
             _rec("loss_grad", 1, ms=0.024)]
    out = bench.summarize_records(recs, maxit=20)
    pcg = out[f"pcg_step@{NB_C2}n"]
    assert pcg["launches"] == 19 and pcg["us_mean"] == pytest.approx(20.0)
    assert pcg["achieved_GBps"] == pytest.approx(108_051_840 / 20e-6 / 1e9, rel=1e-3)
    assert pcg["frac"] == pytest.approx(pcg["achieved_GBps"] / 8000.0, abs=1e-4)
    assert out[f"trial@{NB_C2}n"]["launches"] == 1
    assert out[f"loss_grad@{NB_C2}n"]["launches"] == 1
    step = out[f"loss_grad@{NB_C2}n+step"]
    assert step["launches"] == 2 and step["us_median"] == pytest.approx(23.0)


def test_solver_leg_kernels_at_the_finest_level():
    """Hartley passes as direct sums (2 n flops per node and pass), the block PCG's 16 B/node,
    and the L-BFGS direction's bytes per step from the pairs each step used."""
    coarse = NB_C2 // 8
    recs = [_rec("dht", 3 + 4 * 144, ms=0.030), _rec("dht", 2 + 4 * 111, ms=0.020),
            _rec("dht", 2 + 4 * 72, ms=0.010, nodes=coarse), _rec("block_pcg", 20, ms=0.1),
            _rec("loss_grad", 0)]
    k = bench.leg_kernels("admm", recs, None)
    fl = 2 * 144 * NB_C2 + 2 * 111 * NB_C2
    assert k["dht"]["launches"] == 2 and k["dht"]["flops_per_launch"] == fl // 2
    assert k["dht"]["achieved"] == pytest.approx(fl / 50e-6 / 1e12, rel=1e-3)
    assert k["dht"]["frac"] == pytest.approx(k["dht"]["achieved"] / 157.3, rel=1e-3)
    assert k["block_pcg"]["bytes_per_launch"] == 16 * NB_C2
    assert k["block_pcg"]["achieved"] == pytest.approx(16 * NB_C2 / 100e-6 / 1e9, rel=1e-3)
    # three launches per L-BFGS step; step 0 reads g only, then 20 + 8 p and 8 + 8 c B/node
    lb = [_rec("lbfgs", ph, ms=0.01) for _ in range(3) for ph in range(3)]
    stats = [[], [dict(pcg_iters=0.0), dict(pcg_iters=1.0), dict(pcg_iters=2.0)]]
    d = bench.leg_kernels("lbfgs", lb, stats)["direction"]
    want = [4 + 8, (20 + 0) + (8 + 8), (20 + 8) + (8 + 16)]
    assert [st["bytes"] for st in d["per_step"]] == [w * NB_C2 for w in want]
    assert d["us_mean_per_step"] == pytest.approx(30.0)
    assert d["achieved"] == pytest.approx(sum(want) * NB_C2 / 90e-6 / 1e9, rel=1e-3)
    # a stopped solve (NaN records) or a launch count that does not match gives no figure
    stats_nan = [[], [dict(pcg_iters=float("nan"))] * 3]
    assert "direction" not in bench.leg_kernels("lbfgs", lb, stats_nan)
    assert "direction" not in bench.leg_kernels("lbfgs", lb[:-1], stats)
    q = bench.leg_kernels("lsq", [_rec("lsq", 0, ms=0.27)], None)["lsq"]
    assert q["bytes_per_launch"] == 12 * N_C2 + 4 * NB_C2


def test_batch_level_bytes_sum_the_per_pair_rules():
    from synth.phantom import batch_specs
    lv = bench.batch_level_bytes(n=3)
    assert [r["level"] for r in lv] == [0, 1, 2]
    for r in lv:
        N = Nb = 0
        for sp in batch_specs(3):
            s = tuple(sp["shape"])
            for _ in range(r["level"]):
                s = tuple((x + 1) // 2 for x in s)
            N += int(np.prod(s))
            Nb += int(np.prod([x + (d == sp["pe"]) for d, x in enumerate(s)]))
        assert (r["cells"], r["nodes"]) == (N, Nb)
        assert r["pcg_step"] == 40 * Nb
        assert r["loss_grad"] == 4 * N + 24 * Nb
        assert r["trial"] == 4 * N + 8 * Nb
    assert lv[0]["nodes"] > 7 * lv[1]["nodes"] > 49 * lv[2]["nodes"]


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    copy_kib = bench.COPY_MIB * 1024.0
    for counter, copy_val, pcg_val in (("FETCH_SIZE", copy_kib / 2, 40000.0),
                                       ("WRITE_SIZE", copy_kib, 42000.0)):
        rows = [dict(Dispatch_Id=1, Kernel_Name="void at::native::vectorized_elementwise_kernel",
                     Grid_Size=1 << 26, Counter_Name=counter, Counter_Value=copy_val),
                dict(Dispatch_Id=2, Kernel_Name="void at::native::FillFunctor elementwise",
                     Grid_Size=1 << 26, Counter_Name=counter, Counter_Value=1.0)]
        # iteration 0, 19 full iterations, the last update
        vals = [1.0] + [pcg_val] * 19 + [2.0]
        for i, v in enumerate(vals):
            rows.append(dict(Dispatch_Id=10 + i, Kernel_Name="void rgp::k_pcg_step<float>",
                             Grid_Size=114688, Counter_Name=counter, Counter_Value=v))
        _write_csv(str(tmp_path / counter / "run_counter_collection.csv"), rows)
    with redirect_stdout(io.StringIO()):
        bench.traffic_summary(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"))
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["scale_fetch"] == pytest.approx(2.0) and rec["scale_write"] == pytest.approx(1.0)
    assert rec["launches"] == 19
    assert rec["fetch_bytes"] == round(40000.0 * 2.0 * 1024)
    assert rec["write_bytes"] == round(42000.0 * 1024)
    assert rec["algorithmic_bytes"] == 40 * NB_C2
    assert rec["source_sha256"] == bench.kernel_source_hash()


def _trace_row(name, grid, t0, dur_ns, wg=256):
    return dict(Kernel_Name=name, Grid_Size_X=grid, Workgroup_Size_X=wg, Start_Timestamp=t0,
                End_Timestamp=t0 + dur_ns)


def test_profile_summary_reports_interior_pcg_launches(tmp_path):
    rows, t = [], 0
    for solve in range(2):
        rows.append(_trace_row("void rgp::k_loss_grad<float>(args)", 196608, t, 20000))
        t += 30000
        for i in range(21):  # iteration 0 and the last update are slow here, the rest 24 us
            dur = 50000 if i in (0, 20) else 24000
            rows.append(_trace_row("void rgp::k_pcg_step<float, 1>(args)", 114688, t, dur))
            t += 60000
    _write_csv(str(tmp_path / "run_kernel_trace.csv"), rows)
    _write_csv(str(tmp_path / "run_kernel_stats.csv"),
               [dict(Name="void rgp::k_pcg_step<float, 1>(args)", Calls=42, AverageNs=25000,
                     TotalDurationNs=1050000, Percentage=90.0)])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.profile_summary(str(tmp_path))
    text = buf.getvalue()
    interior = text.split("full iterations only")[1].splitlines()[2].split()
    assert interior[0] == "114688" and interior[1] == "38"
    assert float(interior[2]) == pytest.approx(24.0) and float(interior[3]) == pytest.approx(24.0)


def test_batch_profile_summary_rates_against_level_bytes(tmp_path):
    lv = bench.batch_level_bytes()
    rows, t = [], 0
    durs = {4677632: 640000, 2707456: 120000, 1064960: 45000}   # ns, one grid per level
    for grid, d in durs.items():
        for _ in range(5):
            rows.append(_trace_row("void rgp::k_pcg_step_batch<float, 256, 1, 2, 1>(args)", grid,
                                   t, d))
            t += d + 1000
    rows.append(_trace_row("void rgp::k_trial_batch<bf16_t, float, 2, 9, 256>(args)", 9, t, 5))
    _write_csv(str(tmp_path / "run_kernel_trace.csv"), rows)
    with redirect_stdout(io.StringIO()):
        out = bench.batch_profile_summary(str(tmp_path))
    pcg = [r for r in out if r["kernel"] == "pcg_step"]
    assert [r["grid"] for r in pcg] == sorted(durs, reverse=True)
    for r in pcg:
        assert r["n"] == 5
        assert r["GBps"] == pytest.approx(lv[r["level"]]["pcg_step"] / (durs[r["grid"]] * 1.0),
                                          rel=1e-3)
    assert not [r for r in out if r["kernel"] == "trial"]  # multi-candidate passes are skipped


def test_range_summary_attributes_launches_to_levels_and_steps(tmp_path):
    # one eager correction of 2 levels (level 1 first), 2 Gauss-Newton steps each with 3 launches
    # (enqueue 10 us apart, kernels of 4 us each, 5 us apart), and one correction recorded into a
    # graph (ranges, no launches), which the summary leaves out
    marks, api, kern = [], [], []
    cid, t = 0, 1_000_000

    def rng(name, a, b):
        marks.append(dict(Domain="MARKER_CORE_RANGE_API", Function=name, Process_Id=1,
                          Thread_Id=1, Correlation_Id=0, Start_Timestamp=a, End_Timestamp=b))

    c0 = t
    for lv in (1, 0):
        l0 = t
        for k in range(2):
            s0 = t
            for j in range(3):
                cid += 1
                api.append(dict(Domain="HIP_RUNTIME_API_EXT", Function="hipLaunchKernel",
                                Process_Id=1, Thread_Id=1, Correlation_Id=cid,
                                Start_Timestamp=t + 1000, End_Timestamp=t + 2000))
                gs = 50_000_000 + cid * 9000
                kern.append(dict(Correlation_Id=cid, Kernel_Name="k", Start_Timestamp=gs,
                                 End_Timestamp=gs + 4000))
                t += 10_000
            rng(f"rgp: Gauss-Newton step {k}", s0, t)
        rng(f"rgp: level {lv}", l0, t)
    rng("rgp: correction", c0, t)
    g0 = t + 1000
    rng("rgp: Gauss-Newton step 0", g0 + 10, g0 + 20)
    rng("rgp: level 0", g0, g0 + 30)
    rng("rgp: correction", g0, g0 + 40)
    _write_csv(str(tmp_path / "run_marker_api_trace.csv"), marks)
    _write_csv(str(tmp_path / "run_hip_api_trace.csv"), api)
    _write_csv(str(tmp_path / "run_kernel_trace.csv"), kern)
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.range_summary(str(tmp_path))
    rows = [ln.split() for ln in buf.getvalue().splitlines()[2:]]
    assert [r[:4] for r in rows] == [["2", "1", "2", "3.0"], ["2", "0", "2", "3.0"]]
    for r in rows:
        # host 30 us per step; GPU span 2 x 9 us + 4 us; busy 3 x 4 us
        assert [float(v) for v in r[4:]] == pytest.approx([30.0, 22.0, 12.0])
