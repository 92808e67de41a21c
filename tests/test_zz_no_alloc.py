"""rgp_loss_grad_noalloc (the allocation-free objective/gradient) against rgp_loss_grad.

Both entry points are called through the C ABI (ctypes binding) on the same seeded inputs; the
allocation-free one keeps its block sums in the library's fixed device array, the other in a
caller workspace, and both run the same kernels, so every output must agree bit for bit.  Two
calls in a row, the second on a smaller grid (and another PE axis), check that the array's
contents left by the first call do not leak into the second.  The oracle is checked too, to the
objective and gradient bars.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import rgp as orc
from tests.gpu_helpers import J_RTOL, VEC_RTOL, rel2, rounded, say, smooth_field, to_dev, to_host

pytestmark = pytest.mark.gpu

REAL = {"f64": torch.float64, "f32": torch.float32}
IMG = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _rgp():
    from paper_2403_10706_amd import rgp
    rgp.load()
    return rgp


def _inputs(shape, pe, seed, img, real):
    cfg = dict(synth.WORKLOADS["c1"])
    cfg.update(shape=tuple(shape), pe=pe, seed=seed)
    cfg["bmax"] = max(0.5, min(3.0, shape[pe] / 8.0))
    cfg["lobe_tau"] = (max(2.0, shape[pe] / 5.0), max(3.0, shape[pe] / 3.0))
    p = synth.make_pair(cfg.pop("shape"), cfg.pop("pe"), **cfg)
    Ip, Im = rounded(p.I_plus, IMG[img]), rounded(p.I_minus, IMG[img])
    b = rounded(smooth_field(shape, pe, seed=seed + 1, amp=min(2.0, shape[pe] / 4)), REAL[real])
    return Ip, Im, b


@pytest.mark.parametrize("img,real", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32")])
def test_loss_grad_noalloc_matches_workspace_entry_point(img, real):
    rgp = _rgp()
    dt, it = REAL[real], IMG[img]
    h = (1.0, 1.3, 0.8)
    # first call: a grid large enough for the largest loss_grad launch plan (many blocks of
    # sums); second call: a smaller grid with another PE axis, so it reduces fewer block sums
    # than the first left in the array
    for shape, pe, seed in (((96, 120, 80), 1, 31), ((21, 45, 37), 0, 41)):
        say(f"[noalloc] img={img} real={real} shape={shape} pe={pe}")
        Ip, Im, b = _inputs(shape, pe, seed, img, real)
        Ipd, Imd, bd = to_dev(Ip, it), to_dev(Im, it), to_dev(b, dt)
        ref_j, ref_g, ref_d, ref_o = rgp.loss_grad(Ipd, Imd, bd, pe, h)
        jdsp = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        grad = torch.full_like(bd, float("nan"))
        hd = torch.full_like(bd, float("nan"))
        ho = torch.full_like(bd, float("nan"))
        rgp.loss_grad_noalloc(Ipd, Imd, bd, pe, h, jdsp=jdsp, grad=grad, hdiag=hd, hoff=ho)
        torch.cuda.synchronize()
        assert torch.equal(jdsp, ref_j), (to_host(jdsp), to_host(ref_j))
        assert torch.equal(grad, ref_g)
        assert torch.equal(hd, ref_d)
        assert torch.equal(ho, ref_o)
        # J alone (no field outputs) through the same scratch
        j2 = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        rgp.loss_grad_noalloc(Ipd, Imd, bd, pe, h, jdsp=j2)
        torch.cuda.synchronize()
        assert torch.equal(j2, ref_j)
        # and the oracle, to the parity bars
        obj, gref, _ = orc.objective_gradient(Ip, Im, b, pe, h)
        rt = 1e-12 if real == "f64" else J_RTOL
        assert to_host(jdsp)[0] == pytest.approx(obj.J, rel=rt)
        assert rel2(to_host(grad), gref) <= (1e-11 if real == "f64" else VEC_RTOL)


def test_loss_grad_noalloc_barrier_and_errors():
    """A field outside the barrier gives J = +inf as with the workspace entry point; argument
    errors come back synchronously and enqueue nothing."""
    rgp = _rgp()
    shape, pe = (20, 24, 18), 1
    Ip, Im, b = _inputs(shape, pe, 5, "f32", "f32")
    b = b.copy()
    b[4, 6, 3] += 3.0
    Ipd, Imd, bd = to_dev(Ip, torch.float32), to_dev(Im, torch.float32), to_dev(b, torch.float32)
    jdsp = torch.zeros(4, dtype=torch.float64, device="cuda")
    rgp.loss_grad_noalloc(Ipd, Imd, bd, pe, jdsp=jdsp)
    ref_j, _, _, _ = rgp.loss_grad(Ipd, Imd, bd, pe, want_grad=False, want_hess=False)
    torch.cuda.synchronize()
    assert np.isinf(to_host(jdsp)[0]) and torch.equal(jdsp, ref_j)
    with pytest.raises(rgp.RGPError) as e:   # hdiag without hoff
        rgp.loss_grad_noalloc(Ipd, Imd, bd, pe, jdsp=jdsp, hdiag=torch.empty_like(bd))
    assert e.value.code == -1
