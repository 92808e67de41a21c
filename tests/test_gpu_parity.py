"""GPU-vs-oracle parity of every C-ABI entry point, called through the ctypes binding.

Inputs are seeded and synthetic; the oracle receives the same values the device sees (images and
fields rounded to the device storage type, then FP64).  Tolerances are the bars stated in
``gpu_helpers``; FP64 device runs are additionally held to near-rounding agreement.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import rgp as orc
from tests.gpu_helpers import (B0_ATOL, BFINAL_ATOL, J_RTOL, VEC_RTOL, rel2, rounded, say,
                               smooth_field, to_dev, to_host)

pytestmark = pytest.mark.gpu

REAL = {"f64": torch.float64, "f32": torch.float32}
# (shape, pe): several column tiles and ragged tails along every axis, all three PE axes.
SHAPES = [((32, 32, 24), 1), ((37, 29, 23), 0), ((21, 45, 67), 1), ((19, 26, 41), 2),
          ((70, 9, 130), 0), ((5, 3, 2), 2)]


def _rgp():
    from paper_2403_10706_amd import rgp
    rgp.load()
    return rgp


def _pair(shape, pe, seed, scale=1.0):
    cfg = dict(synth.WORKLOADS["c1"])
    cfg.update(shape=tuple(shape), pe=pe, seed=seed)
    cfg["bmax"] = max(0.5, min(3.0, shape[pe] / 8.0))
    cfg["lobe_tau"] = (max(2.0, shape[pe] / 5.0), max(3.0, shape[pe] / 3.0))
    return synth.make_pair(cfg.pop("shape"), cfg.pop("pe"), scale=scale, **cfg)


def _tol(real, f64, f32):
    return f64 if real == "f64" else f32


@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("shape,pe", SHAPES)
def test_loss_grad_hvp_parity(shape, pe, real):
    rgp = _rgp()
    say(f"[loss_grad/hvp] shape={shape} pe={pe} real={real}")
    p = _pair(shape, pe, seed=11)
    dt = REAL[real]
    h = (1.0, 1.3, 0.8)
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    b = rounded(smooth_field(shape, pe, seed=5, amp=min(2.0, shape[pe] / 4)), dt)
    jdsp, g, hd, ho = rgp.loss_grad(to_dev(Ip, dt), to_dev(Im, dt), to_dev(b, dt), pe, h)
    obj, gref, lin = orc.objective_gradient(Ip, Im, b, pe, h)
    j = to_host(jdsp)
    rt = _tol(real, 1e-12, J_RTOL)
    for got, want in zip(j, (obj.J, obj.D, obj.S, obj.P)):
        assert got == pytest.approx(want, rel=rt, abs=1e-300), (j, obj)
    assert rel2(to_host(g), gref) <= _tol(real, 1e-11, VEC_RTOL)
    dref = orc.gn_diag(lin, pe)
    assert rel2(to_host(hd), dref) <= _tol(real, 1e-12, VEC_RTOL)
    v = np.random.default_rng(3).standard_normal(b.shape)
    v = rounded(v, dt)
    Hv, vhv = rgp.gn_hvp(hd, ho, to_dev(v, dt), shape, pe, h)
    Href = orc.gn_matvec(lin, v, pe)
    assert rel2(to_host(Hv), Href) <= _tol(real, 1e-11, VEC_RTOL)
    assert to_host(vhv)[0] == pytest.approx(float(np.sum(v * Href)), rel=_tol(real, 1e-10, 1e-4))


@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("shape,pe", SHAPES[:5])
def test_pcg_parity(shape, pe, real):
    rgp = _rgp()
    say(f"[pcg] shape={shape} pe={pe} real={real}")
    p = _pair(shape, pe, seed=12)
    dt = REAL[real]
    h = (1.0, 1.0, 1.0)
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    b = rounded(smooth_field(shape, pe, seed=6, amp=min(2.0, shape[pe] / 4)), dt)
    _, g, hd, ho = rgp.loss_grad(to_dev(Ip, dt), to_dev(Im, dt), to_dev(b, dt), pe, h)
    _, gref, lin = orc.objective_gradient(Ip, Im, b, pe, h)
    rhs = -to_host(g)   # the device gradient, rounded to the device type, is the right-hand side
    for maxit, rtol in ((10, 0.0), (25, 0.0), (50, 0.1)):
        x, it, rr = rgp.pcg_solve(hd, ho, to_dev(rhs, dt), shape, pe, h, maxit=maxit, rtol=rtol)
        ref = orc.pcg_solve(lin, rhs, pe, maxit, rtol)
        its = int(to_host(it)[0])
        assert its == ref.iters, (its, ref.iters)
        # FP32 CG drifts from FP64 CG as rounding differences are amplified iteration by
        # iteration (loss of orthogonality): the bar grows linearly beyond 10 iterations
        # (FP64 on the device matches to 1e-9).
        assert rel2(to_host(x), ref.x) <= _tol(real, 1e-9, VEC_RTOL * max(1.0, its / 10.0))
        # the device tracks |r| by the FP64 recurrence over FP32 vectors: compare the normalised
        # residual absolutely in FP32
        got = float(to_host(rr)[0])
        if real == "f64":
            assert got == pytest.approx(ref.relres, rel=1e-6)
        else:
            assert abs(got - ref.relres) <= 1e-4


def test_pcg_zero_rhs_gives_zero():
    rgp = _rgp()
    shape, pe = (12, 14, 10), 1
    p = _pair(shape, pe, seed=13)
    dt = torch.float32
    b = smooth_field(shape, pe, seed=7, amp=1.0)
    _, g, hd, ho = rgp.loss_grad(to_dev(p.I_plus, dt), to_dev(p.I_minus, dt), to_dev(b, dt), pe)
    x, it, rr = rgp.pcg_solve(hd, ho, torch.zeros_like(g), shape, pe, maxit=5, rtol=0.0)
    assert int(to_host(it)[0]) == 0 and float(torch.abs(x).max()) == 0.0


@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("shape,pe", SHAPES)
def test_ot_init_parity(shape, pe, real):
    rgp = _rgp()
    say(f"[ot_init] shape={shape} pe={pe} real={real}")
    p = _pair(shape, pe, seed=14)
    dt = REAL[real]
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    h = (1.0, 1.0, 1.25)
    for guard in (True, False):
        b0, ng = rgp.ot_init(to_dev(Ip, dt), to_dev(Im, dt), pe, h, guard=guard)
        ref = orc.ot_init(Ip, Im, pe, h, eps=1e-3, guard=guard)
        err = float(np.max(np.abs(to_host(b0) - ref.b0)))
        assert err <= B0_ATOL, err
        if guard:
            assert int(to_host(ng)[0]) == ref.guarded_cells


def test_ot_guard_and_empty_columns():
    rgp = _rgp()
    m = 30
    ip = np.full((3, 5, m), 1e-3)
    im = np.full((3, 5, m), 1e-3)
    ip[:, :, 10] = 50.0
    im[:, :, 14] = 50.0
    ip[1, 2, :] = 0.0
    im[1, 2, :] = 0.0
    dt = torch.float64
    for guard in (True, False):
        b0, ng = rgp.ot_init(to_dev(ip, dt), to_dev(im, dt), 2, guard=guard)
        ref = orc.ot_init(ip, im, 2, (1.0, 1.0, 1.0), guard=guard)
        assert float(np.max(np.abs(to_host(b0) - ref.b0))) <= 1e-9
        if guard:
            assert int(to_host(ng)[0]) == ref.guarded_cells > 0
    z = torch.zeros((4, 6, 5), dtype=torch.float32, device="cuda")
    b0, _ = rgp.ot_init(z, z, 1)
    assert float(torch.abs(b0).max()) == 0.0


@pytest.mark.parametrize("img", ["f64", "f32", "bf16"])
def test_apply_correction_parity(img):
    rgp = _rgp()
    shape, pe = (33, 40, 27), 1
    p = _pair(shape, pe, seed=15)
    it = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[img]
    rt = torch.float64 if img == "f64" else torch.float32
    Ip, Im = rounded(p.I_plus, it), rounded(p.I_minus, it)
    b = rounded(smooth_field(shape, pe, seed=8, amp=3.0), rt)
    Tp, Tm = rgp.apply_correction(to_dev(Ip, it), to_dev(Im, it), to_dev(b, rt), pe)
    refp = orc.transform(Ip, b, pe, (1.0, 1.0, 1.0), +1.0)
    refm = orc.transform(Im, b, pe, (1.0, 1.0, 1.0), -1.0)
    tol = {"f64": 1e-13, "f32": 1e-5, "bf16": 1e-2}[img]
    assert rel2(to_host(Tp), refp) <= tol and rel2(to_host(Tm), refm) <= tol
    zero = torch.zeros(tuple(b.shape), dtype=rt, device="cuda")
    Tp, Tm = rgp.apply_correction(to_dev(Ip, it), to_dev(Im, it), zero, pe)
    assert np.array_equal(to_host(Tp), Ip) and np.array_equal(to_host(Tm), Im)


def test_barrier_violation_gives_infinite_objective():
    rgp = _rgp()
    shape, pe = (10, 12, 9), 1
    p = _pair(shape, pe, seed=16)
    b = smooth_field(shape, pe, seed=9, amp=1.0)
    b[3, 5, 4] += 2.0
    jdsp, _, _, _ = rgp.loss_grad(to_dev(p.I_plus, torch.float64), to_dev(p.I_minus, torch.float64),
                                  to_dev(b, torch.float64), pe)
    j = to_host(jdsp)
    ref = orc.objective(p.I_plus, p.I_minus, b, pe, (1.0, 1.0, 1.0))
    assert math.isinf(j[0]) and math.isinf(j[3]) and math.isinf(ref.J)
    assert j[1] == pytest.approx(ref.D, rel=1e-12)


def test_loss_grad_is_deterministic():
    rgp = _rgp()
    p = synth.make_workload("c2")
    dt = torch.float32
    b = smooth_field(p.shape, p.pe, seed=10, amp=4.0)
    args = (to_dev(p.I_plus, dt), to_dev(p.I_minus, dt), to_dev(b, dt), p.pe)
    r1 = rgp.loss_grad(*args)
    r2 = rgp.loss_grad(*args)
    for a, c in zip(r1, r2):
        assert torch.equal(a, c)


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_correct_single_level_c1(real):
    """The small FP64 workload: OT then 5 GN-PCG steps (PCG 10, rtol 0) on one level."""
    rgp = _rgp()
    say(f"[correct c1] real={real}")
    p = synth.make_workload("c1")
    dt = REAL[real]
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    opts = rgp.Options(levels=1, gn_iters=5, pcg_iters=10, pcg_rtol=0.0)
    out = rgp.correct(to_dev(Ip, dt), to_dev(Im, dt), p.pe, opts=opts)
    ref = orc.solve(Ip, Im, p.pe, levels=1, gn_iters=5, pcg_iters=10, pcg_rtol=0.0)
    err = float(np.max(np.abs(to_host(out["b"]) - ref.b)))
    assert err <= _tol(real, 1e-8, BFINAL_ATOL), err
    head, recs = rgp.parse_stats(out["stats"], 1, 5)
    for got, want in zip(recs[0], ref.levels[0][2]):
        assert got["J"] == pytest.approx(want.J, rel=_tol(real, 1e-10, J_RTOL))
        assert got["accepted"] == 1.0 and got["trials"] == want.trials
        assert got["pcg_iters"] == want.pcg_iters
    assert head["ot_guarded"] == ref.ot_guarded
    assert rel2(to_host(out["T_plus"]), ref.T_plus) <= _tol(real, 1e-10, 1e-4)
    assert rel2(to_host(out["T_minus"]), ref.T_minus) <= _tol(real, 1e-10, 1e-4)


@pytest.mark.parametrize("shape,pe,levels", [((40, 48, 36), 1, 2), ((45, 30, 26), 0, 3),
                                             ((20, 22, 50), 2, 2)])
def test_correct_multilevel(shape, pe, levels):
    rgp = _rgp()
    say(f"[correct multilevel] shape={shape} pe={pe} levels={levels}")
    p = _pair(shape, pe, seed=17, scale=30.0)
    dt = torch.float32
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    opts = rgp.Options(levels=levels, gn_iters=4, pcg_iters=8, pcg_rtol=0.0)
    out = rgp.correct(to_dev(Ip, dt), to_dev(Im, dt), pe, opts=opts)
    ref = orc.solve(Ip, Im, pe, levels=levels, gn_iters=4, pcg_iters=8, pcg_rtol=0.0)
    err = float(np.max(np.abs(to_host(out["b"]) - ref.b)))
    assert err <= BFINAL_ATOL, err
    _, recs = rgp.parse_stats(out["stats"], levels, 4)
    for lv in range(levels):
        for got, want in zip(recs[lv], ref.levels[lv][2]):
            assert got["J"] == pytest.approx(want.J, rel=J_RTOL)


def test_correct_with_b_init_zero_iterations_is_identity():
    rgp = _rgp()
    shape, pe = (16, 18, 12), 0
    p = _pair(shape, pe, seed=18)
    dt = torch.float64
    b0 = torch.zeros(rgp.field_shape(shape, pe), dtype=dt, device="cuda")
    opts = rgp.Options(levels=1, gn_iters=0)
    out = rgp.correct(to_dev(p.I_plus, dt), to_dev(p.I_minus, dt), pe, opts=opts, b_init=b0)
    assert torch.equal(out["b"], b0)
    assert np.array_equal(to_host(out["T_plus"]), p.I_plus)
    assert np.array_equal(to_host(out["T_minus"]), p.I_minus)


@pytest.mark.timeout(900)
def test_correct_c2_full_schedule():
    """144x168x111, FP32, 3 levels x 10 GN x 20 PCG (rtol 0): final field within 0.01 voxel."""
    rgp = _rgp()
    say("[correct c2 full schedule] computing on the device")
    p = synth.make_workload("c2")
    dt = torch.float32
    Ip, Im = rounded(p.I_plus, dt), rounded(p.I_minus, dt)
    opts = rgp.Options(levels=3, gn_iters=10, pcg_iters=20, pcg_rtol=0.0)
    out = rgp.correct(to_dev(Ip, dt), to_dev(Im, dt), p.pe, opts=opts)
    b = to_host(out["b"])
    say("[correct c2 full schedule] oracle (about a minute)")
    ref = orc.solve(Ip, Im, p.pe, levels=3, gn_iters=10, pcg_iters=20, pcg_rtol=0.0)
    err = float(np.max(np.abs(b - ref.b)))
    say(f"[correct c2 full schedule] max|b - b_oracle| = {err:.3e} voxel")
    assert err <= BFINAL_ATOL
    _, recs = rgp.parse_stats(out["stats"], 3, 10)
    assert recs[-1][-1]["J"] == pytest.approx(ref.levels[-1][2][-1].J, rel=J_RTOL)


def test_correct_plan_replays_match_eager():
    """The captured graph replays the whole correction; every replay equals the eager result
    bitwise (deterministic reductions), with eager work and synchronisation in between, and a
    replay after the inputs changed in place follows the new inputs."""
    rgp = _rgp()
    shape, pe = (40, 48, 36), 1
    p = _pair(shape, pe, seed=19, scale=30.0)
    dt = torch.float32
    Ip, Im = to_dev(p.I_plus, dt), to_dev(p.I_minus, dt)
    opts = rgp.Options(levels=2, gn_iters=3, pcg_iters=6, pcg_rtol=0.0)
    eager = rgp.correct(Ip, Im, pe, opts=opts)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    nbytes = rgp.workspace_size(rgp.OP_CORRECT, shape, pe, (1.0, 1.0, 1.0), dt, opts.to_c())
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(rgp.field_shape(shape, pe), dtype=dt, device="cuda")
    Tp, Tm = torch.empty_like(Ip), torch.empty_like(Im)
    stats = torch.empty(rgp.STAT_HEADER + 2 * 3 * rgp.STAT_FIELDS, dtype=torch.float64,
                        device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        plan = rgp.Plan(Ip, Im, pe, opts, b, Tp, Tm, ws, stats=stats, stream=s)
        for rep in range(3):
            b.fill_(7.0)
            plan.launch(s)
            s.synchronize()
            assert torch.equal(b, eager["b"]), rep
            assert torch.equal(Tp, eager["T_plus"]) and torch.equal(Tm, eager["T_minus"])
            assert torch.equal(stats, eager["stats"]) or np.allclose(
                to_host(stats), to_host(eager["stats"]), equal_nan=True)
            again = rgp.correct(Ip, Im, pe, opts=opts)   # eager work between replays
            s.synchronize()
            assert torch.equal(again["b"], eager["b"])
        Ip.mul_(1.05)
        Im.mul_(0.97)
        s.synchronize()
        plan.launch(s)
        s.synchronize()
        fresh = rgp.correct(Ip, Im, pe, opts=opts)
        s.synchronize()
        assert torch.equal(b, fresh["b"])
        assert not torch.equal(b, eager["b"])
        plan.close()
