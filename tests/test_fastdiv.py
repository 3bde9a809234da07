"""Host check of the division by a launch-fixed divisor used by the kernels
(csrc/fastdiv.h): compiled with the host C compiler, compared with the
integer division over every divisor up to 4096 on sampled and boundary
dividends below 2^31."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fastdiv_matches_division(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = r'''
#include <stdio.h>
#include "fastdiv.h"
int main(void) {
  unsigned long long bad = 0, n = 0;
  for (uint32_t d = 1; d <= 4096; ++d) {
    FastDiv f = make_fastdiv(d);
    uint32_t xs[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x7fffffffu - 1, 0x40000000u,
                     0x7fffffffu / d * d, 0x7fffffffu / d * d - 1};
    for (unsigned i = 0; i < sizeof(xs) / sizeof(xs[0]); ++i) {
      uint32_t x = xs[i];
      if (x >= 0x80000000u) continue;
      ++n;
      if (fdiv(x, f) != x / d || fmod_(x, f) != x % d) ++bad;
    }
    uint64_t st = 0x9e3779b97f4a7c15ull * d;
    for (int k = 0; k < 2000; ++k) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      uint32_t x = (uint32_t)(st >> 33);
      ++n;
      if (fdiv(x, f) != x / d || fmod_(x, f) != x % d) ++bad;
    }
    for (uint32_t x = 0; x < 70000; ++x) {
      ++n;
      if (fdiv(x, f) != x / d) ++bad;
    }
  }
  printf("%llu %llu\n", n, bad);
  return bad != 0;
}
'''
    (tmp_path / "fd.c").write_text(src)
    subprocess.run([cc, "-O2", "-I", os.path.join(ROOT, "paper_2107_06635_amd", "csrc"), str(tmp_path / "fd.c"),
                    "-o", str(tmp_path / "fd")], check=True)
    out = subprocess.run([str(tmp_path / "fd")], capture_output=True, text=True)
    n, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and n > 1000000, out.stdout
