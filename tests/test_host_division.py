"""Host check of the kernels' division by run constants (pic_device.hpp:
div_magic / div_by, the round-up multiplier of Granlund and Montgomery,
PLDI 1994): the header is compiled for the host and the quotients compared
with C's / over every divisor up to 2048 and the numerators below 2^16, the
multiples k d - 1, k d, k d + 1 across the 32-bit range, and random ones,
including the products nc0 * nc1 that split cell indices."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_15130_amd", "csrc")

PROGRAM = r"""
#include "pic_device.hpp"
#include <cstdio>
#include <random>
using namespace pic;
int main() {
  std::mt19937_64 g(11);
  long bad = 0, checked = 0;
  auto chk = [&](uint32_t d, uint64_t n) {
    if (n > 0xffffffffull) return;
    ++checked;
    if (div_by(div_magic(d), (uint32_t)n) != (uint32_t)n / d) {
      if (bad++ < 5) std::printf("bad d=%u n=%llu\n", d, (unsigned long long)n);
    }
  };
  for (uint32_t d = 1; d <= 2048; ++d) {
    for (uint32_t n = 0; n < (1u << 16); ++n) chk(d, n);
    for (uint64_t k = 1; k < 4096; k += 7) {
      const uint64_t v = k * 1048573ull * d;
      chk(d, v - 1); chk(d, v); chk(d, v + 1);
    }
    chk(d, 0xffffffffull); chk(d, 0x7fffffffull); chk(d, 0x80000000ull);
    for (int r = 0; r < 256; ++r) chk(d, (uint32_t)g());
  }
  for (uint32_t a = 3; a <= 1023; a += 5)
    for (uint32_t b = 3; b <= 1023; b += 61) {
      const uint32_t d = a * b;
      for (int r = 0; r < 64; ++r) chk(d, (uint32_t)g() >> 1);
      for (uint64_t k = 1; k < 64; ++k) { chk(d, k * d - 1); chk(d, k * d); }
    }
  std::printf("checked %ld bad %ld\n", checked, bad);
  return bad != 0;
}
"""


def test_division_by_run_constants_matches_c_division(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "divcheck.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "divcheck"
    subprocess.run([hipcc, "-O2", "--offload-arch=gfx950", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout
    assert "bad 0" in out.stdout and int(out.stdout.split()[1]) > 10**8
