"""Accuracy of the reaction-rate exponential of the HIP path (a 64-entry
2^(j/64) table, Cody-Waite reduction, degree-5 Taylor polynomial): the
device function compiled for the host (hipcc, no GPU needed) against
long-double exp on random arguments and at the ends of the range."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SRC = r'''
#include "physics.h"
#include <cmath>
#include <cstdio>
#include <random>
int main() {
  double tab[64];
  for (int j = 0; j < 64; ++j) tab[j] = (double)exp2l((long double)j / 64.0L);
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u(-700.0, 700.0), v(-40.0, 40.0);
  double worst = 0.0;
  for (long i = 0; i < 400000; ++i) {
    const double x = (i & 1) ? u(g) : v(g);
    const double a = nsdc::exp_tab(x, tab);
    const long double r = expl((long double)x);
    const double ulp = std::nextafter((double)r, INFINITY) - (double)r;
    const double e = (double)fabsl((long double)a - r) / ulp;
    if (e > worst) worst = e;
  }
  printf("%.6f %.17g %.17g %g %g\n", worst, nsdc::exp_tab(0.0, tab), nsdc::exp_tab(1.0, tab),
         nsdc::exp_tab(-746.0, tab), nsdc::exp_tab(710.0, tab));
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_table_exponential_is_within_two_ulp(tmp_path):
    src = tmp_path / "t.hip"
    src.write_text(SRC)
    exe = tmp_path / "t"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I",
                           os.path.join(ROOT, "paper_1309_7327_amd", "csrc"), str(src), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    worst, e0, e1, lo, hi = (float(t) for t in out)
    assert worst < 2.0, worst
    assert e0 == 1.0
    assert abs(e1 - 2.718281828459045) <= 4.5e-16
    assert lo == 0.0 and hi == float("inf")
