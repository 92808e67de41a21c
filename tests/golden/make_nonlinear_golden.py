"""Writes the oracle's whole corrections of full-size pairs in the nonlinear regime, sampled:

* ``c2x1000_solve_sample.npz``: the 3T-brain-shaped pair (144x168x111, PE along dim 1) with the
  images scaled by 1000 and rounded to FP32, 3 levels x 10 GN x 20 PCG (rtol 0).  At this
  intensity scale the distance term outweighs the smoothness term, the recovered field reaches
  several voxels and the line search backtracks;
* ``c5_pair{i}_solve_sample.npz``: pairs i = 1, 6, 29 of the 32-pair uneven batch (sizes,
  PE axes and maximum displacements drawn from the pair's own seed), images scaled by 1000 and
  rounded to BF16, the same schedule.

Each file holds the final field at seeded node positions, its max-abs, the objective, step
size, trial count and acceptance after every Gauss-Newton step, the corrected images at seeded
cell positions, and the OT guard count.

Run from the repository root:  python tests/golden/make_nonlinear_golden.py   (CPU, ~10 min
with the four solves in parallel).  Only the seeded input generator and the oracle are used.
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import rgp as orc  # noqa: E402

LEVELS, GN, PCG = 3, 10, 20
SCALE = 1000.0
NSAMPLE = 16384
C5_PAIRS = (1, 6, 29)
HERE = os.path.dirname(os.path.abspath(__file__))


def _round(x, kind):
    """The values the device sees for x stored as FP32 or BF16 (torch's rounding on the CPU)."""
    import torch
    dt = torch.float32 if kind == "f32" else torch.bfloat16
    return torch.as_tensor(np.ascontiguousarray(x)).to(dt).to(torch.float64).numpy()


def _case(name):
    if name == "c2x1000":
        p = synth.make_workload("c2", scale=SCALE)
        kind = "f32"
    else:
        p = synth.make_batch_pair(int(name.split("pair")[1]), scale=SCALE)
        kind = "bf16"
    return p, kind


def run(name):
    t0 = time.time()
    p, kind = _case(name)
    Ip, Im = _round(p.I_plus, kind), _round(p.I_minus, kind)
    ref = orc.solve(Ip, Im, p.pe, levels=LEVELS, gn_iters=GN, pcg_iters=PCG, pcg_rtol=0.0)
    rng = np.random.default_rng(4096)
    bi = np.sort(rng.choice(ref.b.size, size=min(NSAMPLE, ref.b.size), replace=False))
    ci = np.sort(rng.choice(ref.T_plus.size, size=min(NSAMPLE, ref.T_plus.size), replace=False))
    rec = {k: np.full((LEVELS, GN), np.nan) for k in ("J", "gamma", "trials", "accepted")}
    for lv, (_, _, hist) in enumerate(ref.levels):
        for k, s in enumerate(hist):
            rec["J"][lv, k] = s.J
            rec["gamma"][lv, k] = s.gamma
            rec["trials"][lv, k] = s.trials
            rec["accepted"][lv, k] = float(s.accepted)
    out = os.path.join(HERE, f"{name}_solve_sample.npz")
    np.savez_compressed(out, b_index=bi, b=ref.b.ravel()[bi], cell_index=ci,
                        T_plus=ref.T_plus.ravel()[ci], T_minus=ref.T_minus.ravel()[ci],
                        b_absmax=np.abs(ref.b).max(), ot_guarded=ref.ot_guarded,
                        status=ref.status, shape=np.array(p.shape), pe=p.pe, scale=SCALE,
                        image_type=kind, **rec)
    backtracked = int(np.nansum(rec["trials"] > 1))
    return (f"{out}: {p.shape} pe={p.pe} {kind}, max|b| = {float(np.abs(ref.b).max()):.3f}, "
            f"steps that backtracked: {backtracked}, J final = {rec['J'][-1, -1]:.6e}, "
            f"{time.time() - t0:.0f} s")


def main():
    names = ["c2x1000"] + [f"c5_pair{i}" for i in C5_PAIRS]
    if len(sys.argv) > 1:
        names = sys.argv[1:]
    with mp.Pool(min(len(names), 4)) as pool:
        for line in pool.imap_unordered(run, names):
            print(line, flush=True)


if __name__ == "__main__":
    main()
