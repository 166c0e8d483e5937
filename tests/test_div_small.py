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


AXIS_DRIVER = r"""
#include <stdio.h>
#include <math.h>
#include <algorithm>
using std::min;
using std::max;
#define MLC_MAX_CAND 8
%s
int main(void) {
  long n = 0, bad = 0;
  for (int nc = 2; nc <= 40; ++nc)
    for (int nb = 1; nb <= std::min(nc, 12); ++nb)
      for (int m = 0; m <= 3; ++m)
        for (int ov = 0; ov <= 4; ++ov)
          for (int pou = 0; pou <= 1; ++pou) {
            if (pou == 0 && ov == 0) continue;
            const int N = nc << m;
            for (int g = 1; g < N; ++g) {
              int id[MLC_MAX_CAND];
              double rho[MLC_MAX_CAND], r2[2];
              int b0 = -1;
              const int k = pou_axis_fast(nc, nb, g, m, ov, pou, id, rho);
              const int k2 = pou_axis2(nc, nb, g, m, ov, pou, &b0, r2);
              ++n;
              bool ok = (k > 2) == (k2 > 2);
              if (k <= 2) {
                ok = ok && k2 == k;
                for (int a = 0; a < k; ++a) ok = ok && id[a] == b0 + a && rho[a] == r2[a];
              }
              if (!ok) ++bad;
            }
          }
  printf("%%ld %%ld\n", n, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_gluing_axis_forms_agree(tmp_path):
    """The gluing's loop-free covering blocks (pou_axis2) give the blocks and factors its
    scanning form (pou_axis_fast) finds, for every interior node of grids up to 40 coarse
    cells, 1-12 blocks, overlaps 0-4 and both gluings; both compiled from the kernel source."""
    text = open(SRC).read()
    parts = []
    for name in ("div_small", "pou_axis_fast", "pou_axis2"):
        m = re.search(r"__device__ __forceinline__ (?:int|double) " + name + r"\(.*?\n\}", text, re.S)
        assert m, name + " not found"
        parts.append(m.group(0).replace("__device__ __forceinline__ ", "static inline "))
    c = tmp_path / "axis.cpp"
    c.write_text(AXIS_DRIVER % "\n".join(parts))
    exe = tmp_path / "axis"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    n, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and n > 100_000
