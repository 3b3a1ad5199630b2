"""The kernels' B-spline weight polynomials against the oracle (CPU only).

The kernels evaluate the assignment weights M_p(d + i) and their derivatives
as polynomials in d whose coefficients are generated at compile time
(BsplineCoeffs in the device header).  A small host program built with hipcc
prints those coefficients; they must reproduce the oracle's recursion
(oracle.pppm.bspline) and its derivative (oracle.pppm.dbspline) on [0, 1).
Nothing here runs on a GPU.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import pppm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_15508_amd", "csrc")

DUMP = r"""
#include "device_common.hpp"
#include <cstdio>
template <int P> void dump() {
  constexpr dplr::BsplineCoeffs<P> C{};
  for (int i = 0; i < P; ++i) {
    printf("%d %d", P, i);
    for (int j = 0; j < P; ++j) printf(" %.17g", C.c[i][j]);
    printf("\n");
  }
}
int main() { dump<2>(); dump<3>(); dump<4>(); dump<5>(); dump<6>(); dump<7>(); dump<8>(); return 0; }
"""


@pytest.fixture(scope="module")
def coeffs(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("bspline")
    src, exe = d / "dump.hip", d / "dump"
    src.write_text(DUMP)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    c = {}
    for line in out.split("\n"):
        if line.strip():
            v = line.split()
            c[(int(v[0]), int(v[1]))] = np.array([float(x) for x in v[2:]])
    return c


@pytest.mark.parametrize("p", range(2, 9))
def test_weight_polynomials_match_the_recursion(coeffs, p):
    d = np.linspace(0.0, 1.0, 41, endpoint=False)
    for i in range(p):
        c = coeffs[(p, i)]
        w = np.polynomial.polynomial.polyval(d, c)
        dw = np.polynomial.polynomial.polyval(d, np.polynomial.polynomial.polyder(c))
        assert np.abs(w - pppm.bspline(p, d + i)).max() < 1e-14
        assert np.abs(dw - pppm.dbspline(p, d + i)).max() < 1e-13
