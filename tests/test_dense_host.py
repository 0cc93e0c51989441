"""Host checks of the setup's dense SVD routines (CPU only).

The truncated-SVD Schur complement (``csrc/dense.hpp``) meets Gamma blocks
whose rank is far below their column count; their Householder
bidiagonalisation then runs into vectors many orders below the rounding
level, down to subnormal numbers, and a bidiagonal whose trailing entries
decay past the double range.  This test compiles the native checks with g++
and runs them: reflectors of tiny and subnormal vectors (finite, and mapping
the vector to its norm), convergence of the bidiagonal SVD on graded and
clustered inputs (sum of squares and rotated rows preserved), and the
truncated Schur complement of rank-deficient blocks against an independent
Gram-Schmidt projection.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_dense_svd_routines():
    src = os.path.join(HERE, "native", "dense_svd_test.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "dense_svd_test")
        subprocess.run(["g++", "-std=c++17", "-O1", "-mavx2", "-mfma", "-Wall", "-o", exe, src],
                       check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "dense svd ok" in r.stdout
