"""The C ABI used from C++ alone: the example program (built with the
library) allocates with hipMalloc, runs the FP64 forward product, the
adjoint and the product on the padded SoA layout (AoS -> SoA at the
recommended pitch, the SoA product, back) on a HIP stream, checks the exact
b = I results and a rejected in-place call, and prints "ok"."""

import os
import subprocess

import pytest

from _gpu import say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2103_00571_amd", "examples",
                   "su3_c_api")


@pytest.mark.parametrize("sites", [1, 100003])
def test_c_api_example(sites):
    say("C ABI example sites=%d" % sites)
    assert os.path.exists(EXE), "build the library first (it builds the example too)"
    proc = subprocess.run([EXE, str(sites)], capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert proc.stdout.startswith("ok")
