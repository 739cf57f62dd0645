"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a transposed operand, a wrong sign, a dropped
term, a wrong index, a lost symmetry convention) in a temporary copy of the
oracle's C source, rebuilds it there, and runs the pin tests against the copy:
at least one pin must fail.  Nothing here touches the GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    # (file, original text, mutated text)
    ("oracle_impl.h", "t -= P[k * n + r] * xn[k * d + c];", "t -= P[r * n + k] * xn[k * d + c];"),
    ("oracle_impl.h", "t -= P[r * n + k] * yp[k * d + c];", "t -= P[k * n + r] * yp[k * d + c];"),
    ("oracle_impl.h", "t -= P[r * n + k] * Li[c * n + k];", "t -= P[r * n + k] * Li[k * n + c];"),
    ("oracle_impl.h", "C[r * n + c] -= t;", "C[r * n + c] += t;"),
    ("oracle_impl.h", "return (REAL)(r >= c ? blk[r * n + c] : blk[c * n + r]);",
     "return (REAL)(blk[r * n + c]);"),
    ("oracle_impl.h", "for (int64_t k = r + 1; k < n; ++k) t -= Li[k * n + r] * x[k * d + c];",
     "for (int64_t k = r + 1; k < n; ++k) t -= Li[r * n + k] * x[k * d + c];"),
    ("oracle_impl.h", "if (!(s > 0)) return j + 1;", "if (s < 0) return j + 1;"),
    ("oracle_impl.h", "Lo[r * n + j] = t / ljj;", "Lo[r * n + j] = t * ljj;"),
    ("bds_oracle.c", "dAd[(i * n + r) * n + c] = -0.5 * t;", "dAd[(i * n + r) * n + c] = -1.0 * t;"),
    ("bds_oracle.c", "t += G[((i + 1) * n + r) * d + k] * X[(i * n + c) * d + k] +",
     "t += G[((i + 1) * n + c) * d + k] * X[(i * n + r) * d + k] +"),
    ("bds_oracle.c", "t += s[k * n + r] * X[((i + 1) * n + k) * d + c];",
     "t += s[r * n + k] * X[((i + 1) * n + k) * d + c];"),
    ("bds_oracle.c", "#define REAL long double\n", "#define REAL double\n"),
    ("bds_oracle.c", "out[1] = (double)(l - (long double)out[0]);", "out[1] = 0;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("case", range(len(MUTATIONS)))
def test_planted_mistake_fails_a_pin(case, tmp_path):
    fname, before, after = MUTATIONS[case]
    repo = tmp_path / "repo"
    for sub in ("oracle", "tests", "paper_2509_03015_amd"):
        shutil.copytree(os.path.join(ROOT, sub), repo / sub,
                        ignore=shutil.ignore_patterns("*.so", "*.so.*", "__pycache__", "_lib"))
    path = repo / "oracle" / fname
    src = path.read_text()
    assert src.count(before) == 1, before
    path.write_text(src.replace(before, after))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py"], cwd=repo, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation not caught: {after}\n{r.stdout[-2000:]}"
