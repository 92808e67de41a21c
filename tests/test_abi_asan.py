"""The library's host code under AddressSanitizer (no GPU needed): librgp_asan.so (host code
instrumented with -fsanitize=address, device code as usual) driven by tests/abi_asan_driver.c
through every entry point's argument validation, the workspace sizes of every solver and the
batched plan's dry recording and launch-table merge.  A memory error aborts the driver."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2403_10706_amd")
CLANG = "/opt/rocm/llvm/bin/clang"


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "rgp.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not found")
def test_abi_host_code_under_address_sanitizer(tmp_path):
    from paper_2403_10706_amd import build
    lib = os.path.join(PKG, "librgp_asan.so")
    if _stale(lib):
        build.build(asan=True)
    rt = subprocess.run([CLANG, "-print-resource-dir"], capture_output=True, text=True,
                        check=True).stdout.strip() + "/lib/linux"
    exe = str(tmp_path / "abi_asan")
    subprocess.run([CLANG, "-fsanitize=address", "-shared-libasan", "-g", "-I",
                    os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_asan_driver.c"),
                    "-L", PKG, "-lrgp_asan", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{rt}", "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "all checks passed" in res.stdout
