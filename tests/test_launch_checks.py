"""Host-side bounds of the multi-right-hand-side launches (CPU only).

A matrix-core launch with a split loop writes split x rows x width partial
sums into a buffer sized when the batched buffers were made; the library
checks the product against the buffer before launching and returns
LSAMG_EINVAL instead of overrunning it.  The check is plain C++
(``csrc/launch_checks.hpp``); this test compiles it with g++ and runs its
cases, including a buffer sized for 16 columns reused by a 64-column batch.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_split_capacity_check():
    src = os.path.join(HERE, "native", "launch_checks_test.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "launch_checks_test")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-o", exe, src], check=True)
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "launch checks ok" in r.stdout
