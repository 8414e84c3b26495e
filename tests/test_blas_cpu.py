"""CPU checks of the Fortran-BLAS interposer libozaki_blas.so: it loads,
exports what include/ozaki_blas.h declares, and rejects illegal arguments the
reference-BLAS way (message naming the argument, C untouched) before any
device work."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_interposer_exports_its_header():
    from paper_2603_29975_amd import blas
    lib = blas.library()
    text = open(os.path.join(ROOT, "include", "ozaki_blas.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:void|int)\s+([a-z_0-9]+)\s*\(", text, flags=re.M)
    assert set(names) == {"dgemm_", "zgemm_", "ozaki_blas_config", "ozaki_blas_release"}
    for name in names:
        assert hasattr(lib, name), name
        assert hasattr(blas, name), name


def test_interposer_config_ranges():
    from paper_2603_29975_amd import blas
    assert blas.ozaki_blas_config(13, 0) == -1
    assert blas.ozaki_blas_config(-1, 0) == -1
    assert blas.ozaki_blas_config(0, 1) == -2
    assert blas.ozaki_blas_config(0, 21) == -2
    assert blas.ozaki_blas_config(7, 0) == 0
    assert blas.ozaki_blas_config(0, 14) == 0
    assert blas.ozaki_blas_config(0, 0) == 0


_ARGS_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %r)
from paper_2603_29975_amd import blas
A = np.zeros(64); B = np.zeros(64); C = np.arange(64.0)
cases = [("X", "N", 4, 4, 4, 4, 4, 4), ("N", "Q", 4, 4, 4, 4, 4, 4), ("N", "N", -1, 4, 4, 4, 4, 4),
         ("N", "N", 4, -1, 4, 4, 4, 4), ("N", "N", 4, 4, -1, 4, 4, 4), ("N", "N", 4, 4, 4, 3, 4, 4),
         ("T", "N", 4, 4, 5, 4, 5, 4), ("N", "N", 4, 4, 5, 4, 4, 4), ("N", "C", 4, 5, 4, 4, 4, 4),
         ("N", "N", 4, 4, 4, 4, 4, 3)]
for ta, tb, m, n, k, lda, ldb, ldc in cases:
    blas.dgemm_(ta, tb, m, n, k, 1.0, A, lda, B, ldb, 0.0, C, ldc)
assert np.array_equal(C, np.arange(64.0))
Z = np.zeros(64, dtype=np.complex128)
blas.zgemm_("N", "N", 4, 4, 4, 1.0, Z, 4, Z, 4, 0.0, Z, 2)
blas.dgemm_("N", "N", 0, 4, 4, 1.0, A, 1, B, 4, 0.0, C, 1)        # quick return
blas.dgemm_("N", "N", 4, 4, 4, 0.0, A, 4, B, 4, 1.0, C, 4)        # alpha = 0, beta = 1
assert np.array_equal(C, np.arange(64.0))
print("ok")
"""


def test_interposer_argument_errors_name_the_argument():
    # run in a child process: the messages go to its stderr
    r = subprocess.run([sys.executable, "-c", _ARGS_SCRIPT % ROOT], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().endswith("ok")
    nums = [int(x) for x in re.findall(r"On entry to DGEMM  ?parameter number (\d+)", r.stderr)]
    assert nums == [1, 2, 3, 4, 5, 8, 8, 10, 10, 13], r.stderr
    assert "On entry to ZGEMM  parameter number 13" in r.stderr
