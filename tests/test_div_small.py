"""The gluing kernel's reciprocal quotient (div_small in kernels_grid.hip) is exact: its
source is compiled for the host with gcc and compared with integer division over the
range the kernel uses it for (dividend below 2^22)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1401_4969_amd", "csrc", "kernels_grid.hip")

DRIVER = r"""
#include <stdio.h>
%s
int main(void) {
  long bad = 0, n = 0;
  for (int b = 1; b <= 4096; b += (b < 256 ? 1 : 17)) {
    const float rb = 1.0f / (float)b;
    const int step = b < 16 ? 1 : 97;
    for (int a = 0; a < (1 << 22); a += step) {
      ++n;
      if (div_small(a, b, rb) != a / b) ++bad;
    }
    for (int k = 1; k <= 64; ++k) {  /* every multiple of b near the top, and its neighbours */
      const int a = ((1 << 22) - 1) / b * b - k * b;
      for (int e = -1; e <= 1; ++e)
        if (a + e >= 0 && a + e < (1 << 22)) {
          ++n;
          if (div_small(a + e, b, rb) != (a + e) / b) ++bad;
        }
    }
  }
  printf("%%ld %%ld\n", n, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_div_small_is_exact(tmp_path):
    text = open(SRC).read()
    m = re.search(r"__device__ __forceinline__ int div_small\(int a, int b, float rb\) \{.*?\n\}", text, re.S)
    assert m, "div_small not found"
    body = m.group(0).replace("__device__ __forceinline__ ", "static ")
    c = tmp_path / "div.c"
    c.write_text(DRIVER % body)
    exe = tmp_path / "div"
    subprocess.run(["gcc", "-O2", "-std=c99", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    n, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and n > 10_000_000
