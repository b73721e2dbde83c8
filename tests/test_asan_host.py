"""The library's host code under AddressSanitizer, on the CPU (no GPU needed):
the table construction of pat_plan_create (sensor taps and their per-row
lists, twiddles, shift factors, kappa, PML profiles, built before the first
device allocation, which fails without a GPU) for grids of every kernel
family, and the argument checks of every entry point.  The host side of
pat_api.hip is compiled with the sanitizer (host pass only; the device code
is compiled as usual), linked into a
small C driver (tests/asan/host_checks.c) and run; any sanitizer report or a
wrong status fails the test."""
import os
import shutil
import subprocess

import pytest

from paper_2505_08482_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
CLANG = "/opt/rocm/llvm/bin/clang"


def _have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang not available")
@pytest.mark.skipif(_have_gpu(), reason="the driver expects the device allocation to fail (machine without a GPU)")
def test_host_code_under_address_sanitizer(tmp_path):
    lib = tmp_path / "libpat_asan.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.flags() if f not in ("-O3", "-shared")] + ["-O1", "-g"]
    objs, procs = [], []
    for src in ("pat_api.hip", "batch_launch.hip"):   # the wave solver's host code and its batch launchers
        obj = tmp_path / (src + ".o")
        procs.append(subprocess.Popen([B.hipcc()] + flags + san + ["-c", "-o", str(obj), os.path.join(B.CSRC, src)],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
        objs.append(str(obj))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-2000:]
    subprocess.run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC"] + san + ["-o", str(lib)] + objs,
                   check=True, capture_output=True, timeout=300)
    exe = tmp_path / "host_checks"
    subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address", "-o", str(exe),
                    os.path.join(HERE, "asan", "host_checks.c"), str(lib), f"-Wl,-rpath,{tmp_path}", "-lm"],
                   check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "host checks: 0 failure(s)" in out
