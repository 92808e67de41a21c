"""Writes c3_solve_sample.npz: the oracle's whole correction of the 7T-brain-shaped workload
(200x200x132, PE along dim 0, images rounded to FP32, 4 levels x 10 GN x 20 PCG, rtol 0),
sampled at seeded node and cell positions, with the objective after every GN step.

Run from the repository root:  python tests/golden/make_c3_golden.py   (a few minutes, CPU)
Only the seeded input generator and the oracle are used.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import rgp as orc  # noqa: E402

LEVELS, GN, PCG = 4, 10, 20
NSAMPLE = 8192


def main():
    p = synth.make_workload("c3")
    Ip = p.I_plus.astype(np.float32).astype(np.float64)
    Im = p.I_minus.astype(np.float32).astype(np.float64)
    ref = orc.solve(Ip, Im, p.pe, levels=LEVELS, gn_iters=GN, pcg_iters=PCG, pcg_rtol=0.0)
    rng = np.random.default_rng(2024)
    bi = rng.choice(ref.b.size, size=NSAMPLE, replace=False)
    ci = rng.choice(ref.T_plus.size, size=NSAMPLE, replace=False)
    J = np.array([[s.J for s in hist] for _, _, hist in ref.levels])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_solve_sample.npz")
    np.savez_compressed(out, b_index=bi, b=ref.b.ravel()[bi], cell_index=ci,
                        T_plus=ref.T_plus.ravel()[ci], T_minus=ref.T_minus.ravel()[ci], J=J,
                        b_absmax=np.abs(ref.b).max(), ot_guarded=ref.ot_guarded,
                        shape=np.array(p.shape), pe=p.pe)
    print(out, "max|b| =", float(np.abs(ref.b).max()), "J final =", J[-1, -1])


if __name__ == "__main__":
    main()
