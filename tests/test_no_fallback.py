"""The product path has no CPU fallback: without libsu3.so, or with a
library of another ABI version, the binding and the torch front end refuse
to import. (With the library, CPU tensors are refused rather than computed
on the host: tests/test_abi_cpu.py.)"""

import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_fails_loudly(tmp_path):
    # a copy of the Python package without the built library
    shutil.copytree(os.path.join(ROOT, "paper_2103_00571_amd"), tmp_path / "paper_2103_00571_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    for mod in ("abi", "ops"):
        code = "import sys; sys.path.insert(0, %r); from paper_2103_00571_amd import %s" % (str(tmp_path), mod)
        proc = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
        assert proc.returncode != 0
        assert "ImportError" in proc.stderr and "libsu3.so is not built" in proc.stderr


def test_stale_library_is_refused(tmp_path):
    """A library whose ABI version differs from the binding's is refused."""
    text = open(os.path.join(ROOT, "paper_2103_00571_amd", "abi.py")).read()
    assert "ABI_VERSION = " in text
    shutil.copytree(os.path.join(ROOT, "paper_2103_00571_amd"), tmp_path / "paper_2103_00571_amd",
                    ignore=shutil.ignore_patterns("__pycache__"))
    p = tmp_path / "paper_2103_00571_amd" / "abi.py"
    p.write_text(text.replace("ABI_VERSION = ", "ABI_VERSION = 1000 + ", 1))
    code = "import sys; sys.path.insert(0, %r); from paper_2103_00571_amd import abi" % str(tmp_path)
    proc = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert proc.returncode != 0 and "ImportError" in proc.stderr and "rebuild" in proc.stderr
