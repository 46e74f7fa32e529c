"""The FP64 log-sum-exp helpers of the E-steps (csrc/lse.h), built for the host.

exp_nonpos is held to a 120-bit reference (mpmath) over its whole domain x <= 0,
subnormal results and the underflow to 0 included; lse_push / lse_merge, the
running (max, sum) statistics of eq. 2.4's normalisation, are held to the
log-sum-exp of the same terms in 120-bit arithmetic, with terms far below the
maximum (which the statistics skip) and zero prior weights (a = -inf) mixed in.
"""
import math
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1409_4256_amd", "csrc")

DRIVER = r"""
#include "lse.h"
#include <cstdio>
int main() {
  char mode;
  while (scanf(" %c", &mode) == 1) {
    if (mode == 'e') {  // e x: exp_nonpos(x)
      double x;
      if (scanf("%la", &x) != 1) return 1;
      printf("%a\n", emc::exp_nonpos(x));
    } else {  // s n a_1 .. a_n: statistics of the first half merged with those of the second
      int n;
      if (scanf("%d", &n) != 1) return 1;
      double m1 = -INFINITY, s1 = 0.0, m2 = -INFINITY, s2 = 0.0;
      const emc::ExpCoef ec = emc::exp_coef();
      for (int i = 0; i < n; ++i) {
        double a;
        if (scanf("%la", &a) != 1) return 1;
        if (i < n / 2) emc::lse_push(m1, s1, a, ec); else emc::lse_push(m2, s2, a, ec);
      }
      emc::lse_merge(m1, s1, m2, s2);
      printf("%a %a\n", m1, s1);
    }
  }
}
"""


@pytest.fixture(scope="module")
def lse_bin(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("lse")
    src = d / "lse_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "lse_driver"
    # the header's functions are host-and-device; on the host the attributes are empty
    subprocess.run([cxx, "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-D__forceinline__=inline",
                    "-ffp-contract=off", "-I", CSRC, "-o", str(exe), str(src)], check=True)
    return str(exe)


def _run(exe, text):
    return subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")


def test_exp_nonpos_within_one_unit_over_its_domain(lse_bin):
    mp.mp.prec = 120
    rng = np.random.default_rng(3)
    xs = np.concatenate([
        -rng.uniform(0, 1, 4000), -rng.uniform(0, 64, 8000), -rng.uniform(64, 708, 3000),
        -rng.uniform(708.39, 745.2, 2000),  # subnormal results
        [0.0, -0.0, -5e-324, -1e-300, -1e-17, -math.log(2) / 2, -math.log(2), -64.0, -708.3964185322641,
         -745.1332191019411, -745.2, -746.0, -1e6, -math.inf, math.nan]])
    out = _run(lse_bin, "".join(f"e {float(x).hex()}\n" for x in xs))
    for x, o in zip(xs, out):
        y = float.fromhex(o)
        if not (x >= -745.2):  # below the smallest subnormal's half, -inf and NaN: 0
            assert y == 0.0, (x, y)
            continue
        ref = mp.exp(mp.mpf(float(x)))
        r = float(ref)
        if r == 0.0:
            assert y == 0.0, (x, y)
            continue
        err = float(abs(mp.mpf(y) - ref) / np.spacing(r))
        assert err <= 1.0, (x, y, r, err)
    for i in np.flatnonzero(xs == 0.0):  # exp(+-0) is exactly 1
        assert float.fromhex(out[i]) == 1.0


@pytest.mark.parametrize("case", ["spread", "concentrated", "with_minus_inf", "single", "empty_half"])
def test_running_statistics_equal_the_log_sum_exp(lse_bin, case):
    mp.mp.prec = 120
    rng = np.random.default_rng({"spread": 1, "concentrated": 2, "with_minus_inf": 3, "single": 4,
                                 "empty_half": 5}[case])
    if case == "spread":  # terms over hundreds of units: most far below the maximum
        a = rng.normal(-5000.0, 300.0, 3000)
    elif case == "concentrated":  # all within a few units of each other
        a = rng.normal(1234.5, 2.0, 3000)
    elif case == "with_minus_inf":
        a = rng.normal(0.0, 40.0, 2000)
        a[rng.choice(a.size, 300, replace=False)] = -math.inf
    elif case == "single":
        a = np.array([-77.25])
    else:  # the first half empty (all -inf): the merge takes the second half's statistics
        a = np.concatenate([np.full(10, -math.inf), rng.normal(3.0, 5.0, 11)])
    text = f"s {a.size} " + " ".join(float(v).hex() for v in a) + "\n"
    m, s = (float.fromhex(t) for t in _run(lse_bin, text)[0].split())
    fin = [mp.mpf(float(v)) for v in a if np.isfinite(v)]
    ref = mp.log(mp.fsum(mp.exp(v) for v in fin))
    assert m == max(float(v) for v in fin)
    assert s >= 1.0
    got = mp.mpf(m) + mp.log(mp.mpf(s))
    # the sum carries one rounding per term (relative 2^-53 each, 3000 terms at most)
    assert abs(got - ref) <= 3000 * 2.0 ** -53, (case, float(got - ref))
