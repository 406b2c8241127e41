"""Device code must not write through the scalar data cache: compile every
HIP source of the library to gfx950 assembly and check that no scalar
memory store, scalar atomic or scalar-cache write-back/discard appears
(all stores go through vector memory instructions)."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = sorted(glob.glob(os.path.join(ROOT, "paper_2309_05435_amd", "csrc", "*.hip")))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic_|"
                       r"s_dcache_wb|s_dcache_discard)", re.M)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", SOURCES, ids=os.path.basename)
def test_no_scalar_memory_writes(src, tmp_path):
    out = tmp_path / "k.s"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                    "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                    "-S", "-o", str(out), src], check=True, capture_output=True)
    asm = out.read_text()
    assert "s_endpgm" in asm
    hits = FORBIDDEN.findall(asm)
    assert not hits, f"{os.path.basename(src)}: {sorted(set(hits))}"
