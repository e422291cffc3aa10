"""Device-code hygiene, checked on the gfx950 assembly of every kernel file (CPU only):
no scalar-cache writes (scalar stores, scalar atomics, scalar cache write-back or
discard) and no packed FP32 arithmetic, which the build disables."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2605_13855_amd import build as B  # noqa: E402

CSRC = os.path.join(ROOT, "paper_2605_13855_amd", "csrc")
SCALAR_WRITE = re.compile(r"^\s*s_(store|atomic|buffer_store|buffer_atomic|dcache_wb|dcache_discard|scratch_store)",
                          re.M)
PACKED_F32 = re.compile(r"^\s*v_pk_(add|mul|fma)_f32", re.M)


@pytest.mark.parametrize("src", sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")))
def test_no_scalar_writes_or_packed_fp32(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [B.hipcc(), *B.FLAGS, "--offload-device-only", "-S", os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    asm = out.read_text()
    assert not SCALAR_WRITE.findall(asm), f"{src}: scalar-cache write in device code"
    assert not PACKED_F32.findall(asm), f"{src}: packed FP32 instruction in device code"
