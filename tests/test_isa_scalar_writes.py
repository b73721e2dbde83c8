"""The gfx950 device code of the library performs no memory writes through the
scalar data cache (scalar stores, scalar atomics, scalar-cache write-back):
every store is a vector memory instruction.  Checked on the assembly that
hipcc produces for the library (CPU only; needs hipcc)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2505_08482_amd import build as B

FORBIDDEN = re.compile(
    r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic_|s_dcache_wb|s_dcache_discard)",
    re.M)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
@pytest.mark.parametrize("source", B.SOURCES)
def test_device_code_has_no_scalar_memory_writes(tmp_path, source):
    """Every source linked into the library (the wave solver and the MFMA
    network kernels)."""
    out = tmp_path / (source + ".s")
    flags = [f for f in B.flags() if f not in ("-shared", "-fPIC")]
    cmd = [B.hipcc()] + flags + ["--cuda-device-only", "-S", "-o", str(out),
                                 os.path.join(B.CSRC, source)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    assert "v_" in asm and "global_store" in asm
    bad = sorted(set(m.group(1) for m in FORBIDDEN.finditer(asm)))
    assert not bad, bad
