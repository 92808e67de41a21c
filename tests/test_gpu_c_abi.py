"""The C ABI from a plain C program on the GPU (tests/abi_gpu_driver.c, built by
__graft_entry__.build()): device buffers from hipMalloc, an eager rgp_correct and two replays of
its captured plan, against the same correction through the Python binding."""
import os
import subprocess

import numpy as np
import pytest
import torch

from tests.gpu_helpers import rounded, say, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "_bin", "abi_gpu_driver")


@pytest.mark.parametrize("shape,pe", [((24, 20, 16), 1), ((17, 13, 22), 2), ((19, 26, 11), 0)])
def test_c_program_equals_python_binding(shape, pe, tmp_path):
    """Field of the C program's eager correction (FP32, 2 levels x 3 GN x 8 PCG) equals the
    binding's byte for byte, and the program's plan replays equal its eager result."""
    from paper_2403_10706_amd import rgp
    import synth
    assert os.path.exists(DRIVER), "tests/_bin/abi_gpu_driver is missing: run __graft_entry__.build()"
    rgp.load()
    cfg = dict(synth.WORKLOADS["c1"])
    cfg.update(seed=91)
    cfg["bmax"] = max(0.5, min(3.0, shape[pe] / 8.0))
    cfg["lobe_tau"] = (max(2.0, shape[pe] / 5.0), max(3.0, shape[pe] / 3.0))
    cfg.pop("shape")
    cfg.pop("pe")
    p = synth.make_pair(shape, pe, scale=30.0, **cfg)
    Ip = rounded(p.I_plus, torch.float32).astype(np.float32)
    Im = rounded(p.I_minus, torch.float32).astype(np.float32)
    fp, fm, fb = (str(tmp_path / n) for n in ("ip.f32", "im.f32", "b.f32"))
    np.ascontiguousarray(Ip).tofile(fp)
    np.ascontiguousarray(Im).tofile(fm)
    say(f"[c abi] shape={shape} pe={pe}: running {DRIVER}")
    r = subprocess.run([DRIVER, fp, fm, *map(str, shape), str(pe), "2", "3", "8", fb],
                       capture_output=True, text=True, timeout=120)
    say(r.stdout.strip(), r.stderr.strip())
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert "replays equal eager: yes" in r.stdout
    b_c = np.fromfile(fb, dtype=np.float32).reshape(rgp.field_shape(shape, pe))
    opts = rgp.Options(levels=2, gn_iters=3, pcg_iters=8, pcg_rtol=0.0)
    ref = rgp.correct(to_dev(Ip, torch.float32), to_dev(Im, torch.float32), pe, opts=opts)
    b_py = ref["b"].cpu().numpy()
    say(f"[c abi] max|b_c - b_python| = {float(np.max(np.abs(b_c - b_py))):.3e}")
    assert np.array_equal(b_c, b_py)
