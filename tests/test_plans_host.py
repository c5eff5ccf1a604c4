"""Host-side logic of the kernel plans (plans.hpp, compiled here with the host compiler): the
rows-per-XCD finalize order must be a bijection of the object tiles for every tile grid, and must
keep each tile row on one XCD where the row count allows it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK = r'''
#include <cstdio>
#include <vector>
#define __host__
#define __device__
#include "plans.hpp"
int main() {
  int bad = 0;
  for (int trows = 1; trows <= 70; ++trows)
    for (int tpr = 1; tpr <= 40; ++tpr) {
      const int nt = trows * tpr;
      std::vector<int> seen(nt, 0);
      for (int i = 0; i < nt; ++i) {
        const int t = emg::rows_per_xcd_tile(i, nt, tpr);
        if (t < 0 || t >= nt) { ++bad; continue; }
        ++seen[t];
        // a multiple of 8 tile rows: block i's tile row is on block i's XCD
        if (trows % 8 == 0 && (t / tpr) % 8 != i % 8) ++bad;
      }
      for (int t = 0; t < nt; ++t) bad += seen[t] != 1;
    }
  std::printf("%d\n", bad);
  return bad != 0;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_rows_per_xcd_order_is_a_bijection(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2511_01793_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True, capture_output=True, timeout=120)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout
