"""Neighbour-list entry encoding (pair_code.hpp), checked on the host.

The entry packs a neighbour index and an image shift per axis; the parameter rules
keep every shift the pair searches can produce inside -3 .. 3 (the real-space reach,
cutoff times sqrt(1 + gamma^2) on a sheared lattice, stays below three box lengths,
so the brute-force search's shift bound int(reach / L) + 1 is at most 3).
"""
import math
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2607_25161_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "pair_code.hpp"
int main() {
  const int idx[] = {0, 1, 12345, (1 << 22) - 1};
  int bad = 0;
  for (int j : idx)
    for (int sx = -3; sx <= 3; ++sx)
      for (int sy = -3; sy <= 3; ++sy)
        for (int sz = -3; sz <= 3; ++sz) {
          const uint32_t c = fsd::pack_entry(j, sx, sy, sz);
          if (fsd::entry_index(c) != j || fsd::entry_shift(c, 0) != sx || fsd::entry_shift(c, 1) != sy ||
              fsd::entry_shift(c, 2) != sz)
            ++bad;
        }
  std::printf("%d\n", bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_pack_unpack_round_trip(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-std=c++17", "-D__host__=", "-D__device__=", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "0"


@pytest.mark.parametrize("gam", [0.0, 0.3, -0.5, 0.5])
def test_guard_bounds_the_shift(gam):
    # the largest cutoff the rule accepts gives a brute-force shift bound of 3
    L = 10.0
    le = gam != 0.0
    rcut = math.nextafter(3.0 * L / (math.sqrt(1.25) if le else 1.0), 0.0)
    reach = rcut * math.sqrt(1.0 + gam * gam)
    assert int(reach / L) + 1 <= 3
