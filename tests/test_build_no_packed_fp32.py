"""The built library's gfx950 code holds no packed FP32 arithmetic
(v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32).  The build switches the
packed-fp32-ops target feature off for the device pass; the host pass of
hipcc warns that it does not know the feature, which is harmless, so this
test checks the device code itself: the code object is unbundled from the
library's fat binary and disassembled with the ROCm LLVM tools."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2602_15130_amd", "libpic.so")
LLVM = "/opt/rocm/llvm/bin"


def _tool(name):
    p = os.path.join(LLVM, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not installed")
    return p


def test_device_code_has_no_packed_fp32_arithmetic(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    fat = tmp_path / "fat.bin"
    co = tmp_path / "gfx950.o"
    subprocess.check_call([_tool("llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", LIB,
                           str(tmp_path / "copy.so")])
    subprocess.check_call([_tool("clang-offload-bundler"), "--unbundle", "--type=o",
                           "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fat}",
                           f"--output={co}"])
    dis = subprocess.run([_tool("llvm-objdump"), "-d", "--mcpu=gfx950", str(co)],
                         check=True, capture_output=True, text=True).stdout
    assert dis.count("\n") > 10000 and "k_particles_mixed" in dis
    found = sorted(set(re.findall(r"v_pk_(?:add|mul|fma)_f32", dis)))
    assert not found, found
