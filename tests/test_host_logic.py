"""Host-side logic of libbds that needs no GPU: the refinement stopping rule.

The rule (csrc/bds_refine.hpp) is compiled with g++ into a small driver and
fed correction-norm sequences with known behaviour.
"""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_03015_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cmath>
#include "bds_refine.hpp"
int main() {
    double tol, xn; int n;
    while (std::scanf("%lf %lf %d", &tol, &xn, &n) == 3) {
        double prev = HUGE_VAL; int conv = 0, it = 0;
        for (int k = 0; k < n; ++k) {
            double cn; std::scanf("%lf", &cn);
            if (it == 0 || it == k) {
                ++it;
                if (bds::refine_stop(cn, xn, prev, tol, conv)) { it = -it; }
            }
            if (it < 0) { for (int q = k + 1; q < n; ++q) std::scanf("%lf", &cn); break; }
        }
        std::printf("%d %d\n", it < 0 ? -it : it, conv);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "drv.cpp")
    exe = os.path.join(d, "drv")
    with open(src, "w") as fh:
        fh.write(DRIVER)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", CSRC, src, "-o", exe])
    return exe


def run(driver, tol, xn, seq):
    inp = f"{tol} {xn} {len(seq)} " + " ".join(repr(float(c)) for c in seq) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split()
    return int(out[0]), int(out[1])


def test_geometric_contraction_stops_on_estimated_error(driver):
    # corrections contracting by 6e-4 per step from 6e-4: after the third the
    # estimated remaining error 6e-4 * 2.2e-10 is below 1e-11, after the second it is not
    seq = [6e-4 * (6e-4) ** k for k in range(8)]
    assert run(driver, 1e-11, 1.0, seq) == (3, 1)
    # the plain criterion alone would need the correction itself below tol
    assert run(driver, 1e-14, 1.0, seq) == (4, 1)


def test_first_iteration_uses_plain_criterion(driver):
    assert run(driver, 1e-10, 1.0, [5e-11, 1e-30]) == (1, 1)
    assert run(driver, 1e-10, 1.0, [5e-10, 1e-30]) == (2, 1)


def test_stagnation_stops_and_reports(driver):
    # no contraction: stop at the second iteration; converged only if already tiny
    assert run(driver, 1e-14, 1.0, [1e-3, 9e-4, 8e-4]) == (2, 0)
    assert run(driver, 1e-14, 1.0, [1e-9, 9e-10, 8e-10]) == (2, 1)


def test_nan_stops_unconverged(driver):
    assert run(driver, 1e-14, 1.0, [1e-3, float("nan")]) == (2, 0)


def test_slow_contraction_is_not_trusted(driver):
    # rho = 0.6 >= 0.5: no estimate is used, and the rule stops as non-contracting
    assert run(driver, 1e-11, 1.0, [1e-3, 6e-4, 3.6e-4]) == (2, 0)
