"""C-ABI checks that need no GPU: the library loads, exports every entry point that
``include/rgp.h`` declares, and rejects bad arguments synchronously without touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgp.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[a-z_]+\s*\*?\s+)+\**(rgp_[a-z_]+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2403_10706_amd import rgp
    return rgp.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("rgp_ot_init", "rgp_loss_grad", "rgp_gn_hvp", "rgp_pcg_solve", "rgp_correct"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_2403_10706_amd import rgp
    assert set(_declared()) == set(rgp.EXPORTS)


def test_status_strings_and_defaults(lib):
    from paper_2403_10706_amd import rgp
    assert lib.rgp_status_string(0) == b"ok"
    assert lib.rgp_status_string(-8).startswith(b"workspace")
    # the device-side failures of a correction have their own codes and texts
    texts = {c: lib.rgp_status_string(c) for c in range(-8, 1)}
    assert len(set(texts.values())) == 9 and b"unknown" not in b"".join(texts.values())
    assert (rgp.ENONFINITE, rgp.EBARRIER, rgp.ELINESEARCH) == (-4, -5, -6)
    src = open(HEADER).read()
    for name, code in (("RGP_ENONFINITE", -4), ("RGP_EBARRIER", -5), ("RGP_ELINESEARCH", -6)):
        assert re.search(rf"{name}\s*=\s*{code}\b", src), name
    o = rgp.SolverOpts()
    lib.rgp_default_opts(ctypes.byref(o))
    assert o.alpha == 300.0 and o.beta == 1e-4 and o.pcg_iters == 10 and o.pcg_rtol == 0.1
    assert o.ls_max_trials == 10 and o.ot_guard == 1


def test_workspace_size_and_validation(lib):
    from paper_2403_10706_amd import rgp
    g = rgp.make_grid((144, 168, 111), 1)
    n = ctypes.c_size_t(0)
    for op in range(6):
        o = rgp.SolverOpts()
        lib.rgp_default_opts(ctypes.byref(o))
        o.levels = 3
        assert lib.rgp_workspace_size(op, ctypes.byref(g), rgp.F32, ctypes.byref(o),
                                      ctypes.byref(n)) == 0
        assert n.value > 0 and n.value % 256 == 0
    # the full solve needs the pyramid and ~12 field arrays
    o.levels = 3
    lib.rgp_workspace_size(rgp.OP_CORRECT, ctypes.byref(g), rgp.F32, ctypes.byref(o),
                           ctypes.byref(n))
    nb = 144 * 169 * 111 * 4
    assert n.value >= 12 * nb
    # bad grids / dtypes / options are rejected before any device work
    bad = rgp.make_grid((144, 1, 111), 1)
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -2
    bad = rgp.make_grid((4, 4, 4), 3)
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -1
    bad = rgp.make_grid((4, 4, 4), 1, h=(1.0, 0.0, 1.0))
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -1
    assert lib.rgp_workspace_size(1, ctypes.byref(g), rgp.BF16, None, ctypes.byref(n)) == -3
    # the contiguous field axis holds at most 512 nodes; at most 2^28 field nodes
    ok = rgp.make_grid((16, 16, 512), 1)
    assert lib.rgp_workspace_size(1, ctypes.byref(ok), rgp.F32, None, ctypes.byref(n)) == 0
    bad = rgp.make_grid((16, 16, 513), 1)
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -2
    ok = rgp.make_grid((16, 16, 511), 2)
    assert lib.rgp_workspace_size(1, ctypes.byref(ok), rgp.F32, None, ctypes.byref(n)) == 0
    bad = rgp.make_grid((16, 16, 512), 2)
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -2
    bad = rgp.make_grid((2048, 2048, 128), 0)
    assert lib.rgp_workspace_size(1, ctypes.byref(bad), rgp.F32, None, ctypes.byref(n)) == -2
    o.levels = 0
    assert lib.rgp_workspace_size(rgp.OP_CORRECT, ctypes.byref(g), rgp.F32, ctypes.byref(o),
                                  ctypes.byref(n)) == -1
    o.levels = 9   # 168 cells along PE halve to 1 cell on the ninth level
    assert lib.rgp_workspace_size(rgp.OP_CORRECT, ctypes.byref(g), rgp.F32, ctypes.byref(o),
                                  ctypes.byref(n)) == -2


def test_entry_points_reject_bad_arguments_without_device(lib):
    from paper_2403_10706_amd import rgp
    g = rgp.make_grid((8, 9, 10), 1)
    fake = ctypes.c_void_p(0x1000)
    # missing workspace
    assert lib.rgp_loss_grad(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, fake, 300.0, 1e-4,
                             fake, None, None, None, None, 0, None) == -8
    # missing field
    assert lib.rgp_loss_grad(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, None, 300.0, 1e-4,
                             fake, None, None, None, fake, 1 << 30, None) == -1
    # hdiag without hoff
    assert lib.rgp_loss_grad(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, fake, 300.0, 1e-4,
                             fake, None, fake, None, fake, 1 << 30, None) == -1
    # the allocation-free variant checks the same arguments before it touches the device
    assert lib.rgp_loss_grad_noalloc(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, None, 300.0,
                                     1e-4, fake, None, None, None, None) == -1
    assert lib.rgp_loss_grad_noalloc(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, fake, 300.0,
                                     1e-4, fake, None, fake, None, None) == -1
    assert lib.rgp_loss_grad_noalloc(ctypes.byref(g), rgp.F64, fake, fake, rgp.F32, fake, 300.0,
                                     1e-4, fake, None, None, None, None) == -3
    # FP64 images with FP32 arithmetic is not offered
    assert lib.rgp_loss_grad(ctypes.byref(g), rgp.F64, fake, fake, rgp.F32, fake, 300.0, 1e-4,
                             fake, None, None, None, fake, 1 << 30, None) == -3
    # negative weight
    assert lib.rgp_loss_grad(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, fake, -1.0, 1e-4,
                             fake, None, None, None, fake, 1 << 30, None) == -1
    assert lib.rgp_pcg_solve(ctypes.byref(g), rgp.F32, fake, fake, 300.0, fake, fake, 0, 0.1,
                             None, None, fake, 1 << 30, None) == -1
    assert lib.rgp_ot_init(ctypes.byref(g), rgp.BF16, fake, fake, rgp.BF16, fake, 1e-3, 1, None,
                           fake, 1 << 30, None) == -3
    assert lib.rgp_ot_init(None, rgp.F32, fake, fake, rgp.F32, fake, 1e-3, 1, None, fake,
                           1 << 30, None) == -1
    o = rgp.SolverOpts()
    lib.rgp_default_opts(ctypes.byref(o))
    o.use_b_init = 1
    assert lib.rgp_correct(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, ctypes.byref(o), None,
                           fake, None, None, None, fake, 1 << 30, None) == -1
    o.use_b_init = 0
    o.ls_max_trials = 11
    assert lib.rgp_correct(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, ctypes.byref(o), None,
                           fake, None, None, None, fake, 1 << 30, None) == -1
    # misaligned workspace
    o.ls_max_trials = 10
    assert lib.rgp_correct(ctypes.byref(g), rgp.F32, fake, fake, rgp.F32, ctypes.byref(o), None,
                           fake, None, None, None, ctypes.c_void_p(0x1004), 1 << 30, None) == -8
    # the blur of the OT field works out of place, on FP32 or FP64 fields
    assert lib.rgp_blur_field(ctypes.byref(g), rgp.F32, fake, fake, None) == -1
    assert lib.rgp_blur_field(ctypes.byref(g), rgp.BF16, fake, ctypes.c_void_p(0x2000), None) == -3
    assert lib.rgp_blur_field(None, rgp.F32, fake, ctypes.c_void_p(0x2000), None) == -1
    # pyramid transfers of images: distinct buffers, field-type results, extents >= 1
    assert lib.rgp_restrict_image(ctypes.byref(g), rgp.F32, fake, rgp.F32, fake, None) == -1
    assert lib.rgp_restrict_image(ctypes.byref(g), rgp.F32, fake, rgp.BF16,
                                  ctypes.c_void_p(0x2000), None) == -3
    assert lib.rgp_restrict_image(ctypes.byref(g), rgp.F64, fake, rgp.F32,
                                  ctypes.c_void_p(0x2000), None) == -3
    g0 = rgp.make_grid((0, 4, 4), 1)
    assert lib.rgp_restrict_image(ctypes.byref(g0), rgp.F32, fake, rgp.F32,
                                  ctypes.c_void_p(0x2000), None) == -2
    assert lib.rgp_restrict_image_adjoint(ctypes.byref(g), rgp.BF16, fake,
                                          ctypes.c_void_p(0x2000), 0, None) == -3
    assert lib.rgp_restrict_image_adjoint(ctypes.byref(g), rgp.F64, fake, fake, 1, None) == -1
    assert lib.rgp_restrict_image_adjoint(ctypes.byref(g), rgp.F64, None, fake, 0, None) == -1
    # OT columns beyond the kernel's 8192 cells: RGP_ESHAPE before anything is launched
    gl = rgp.make_grid((9000, 2, 2), 0)
    assert lib.rgp_ot_init(ctypes.byref(gl), rgp.F32, fake, fake, rgp.F32, fake, 1e-3, 1, None,
                           fake, 1 << 30, None) == -2
    gc = rgp.make_grid((40000, 2, 2), 0)  # coarsest of 3 levels: 10000 cells along PE
    o.levels = 3
    assert lib.rgp_correct(ctypes.byref(gc), rgp.F32, fake, fake, rgp.F32, ctypes.byref(o), None,
                           fake, None, None, None, fake, 1 << 30, None) == -2
    o.levels = 4  # coarsest: 5000 cells; the workspace check comes next
    assert lib.rgp_correct(ctypes.byref(gc), rgp.F32, fake, fake, rgp.F32, ctypes.byref(o), None,
                           fake, None, None, None, fake, 16, None) == -8


def test_batch_workspace_size_and_limits(lib):
    from paper_2403_10706_amd import rgp
    opts = rgp.Options(levels=2, gn_iters=2, pcg_iters=3)
    shapes = [(20, 24, 16), (18, 30, 22), (26, 17, 19)]
    pes = [1, 0, 1]
    n_all = rgp.batch_workspace_size(shapes, pes, __import__("torch").float32, opts)
    single = 0
    for sh, pe in zip(shapes, pes):
        single += rgp.workspace_size(rgp.OP_CORRECT, sh, pe, (1.0, 1.0, 1.0),
                                     __import__("torch").float32, opts.to_c())
    assert n_all > single                      # every pair's workspace plus the launch tables
    n = ctypes.c_size_t(0)
    g = (rgp.Grid * 1)(rgp.make_grid((16, 16, 300), 1))   # contiguous axis above 256 nodes
    c = opts.to_c()
    assert lib.rgp_batch_workspace_size(1, g, rgp.F32, ctypes.byref(c), ctypes.byref(n)) == -2
    assert lib.rgp_batch_workspace_size(0, g, rgp.F32, ctypes.byref(c), ctypes.byref(n)) == -1
    c.use_b_init = 1
    g = (rgp.Grid * 1)(rgp.make_grid((16, 16, 20), 1))
    assert lib.rgp_batch_workspace_size(1, g, rgp.F32, ctypes.byref(c), ctypes.byref(n)) == -1
    # the batch's minimum march length: 0..64
    g = (rgp.Grid * 1)(rgp.make_grid((16, 16, 20), 1))
    for march, want in ((0, 0), (16, 0), (64, 0), (-1, -1), (65, -1)):
        c = rgp.Options(levels=2, gn_iters=2, pcg_iters=3, batch_march=march).to_c()
        assert lib.rgp_batch_workspace_size(1, g, rgp.F32, ctypes.byref(c),
                                            ctypes.byref(n)) == want, march
