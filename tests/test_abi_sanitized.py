"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libsu3 is compiled again with the sanitizers on its host code only (each
-fsanitize flag behind -Xarch_host; the GPU code is built as usual) into a
temporary library, and the ABI validation tests (tests/test_abi_cpu.py, no
GPU needed: every call there is rejected or is a no-op before any HIP call)
run against that build in a child process with clang's ASan runtime
preloaded. Any out-of-bounds access, use of freed memory or undefined
arithmetic (signed overflow in a size computation, a bad shift) in the
argument checks stops the run with a report.
"""

import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _clang_asan_runtime():
    pats = ["/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
            "/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"]
    for pat in pats:
        hits = sorted(glob.glob(pat))
        if hits:
            return hits[-1]
    return None


def test_abi_validation_under_sanitizers(tmp_path):
    runtime = _clang_asan_runtime()
    if runtime is None:
        pytest.skip("clang's ASan runtime is not installed")
    from paper_2103_00571_amd import build
    so = build.build(str(tmp_path / "libsu3_san.so"), extra=HOST_SAN)
    # the host code is instrumented: it calls into the ASan and UBSan runtimes
    syms = subprocess.run(["nm", "-D", "--undefined-only", so], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    # the HIP runtime the library links is not instrumented: its own
    # allocations are not ours to judge, and leaks are out of scope
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:alloc_dealloc_mismatch=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["SU3_LIB_PATH"] = so
    env["PYTHONPATH"] = os.pathsep.join([ROOT] + ([env["PYTHONPATH"]] if env.get("PYTHONPATH") else []))
    probe = subprocess.run([sys.executable, "-c", "from paper_2103_00571_amd import abi; print(abi.LIB_PATH)"],
                           env=env, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert probe.returncode == 0 and probe.stdout.strip() == so, (probe.stdout + probe.stderr)[-2000:]
    proc = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_abi_cpu.py"), "-q",
                           "-m", "not gpu", "-k", "not torch_front_end", "-p", "no:cacheprovider"],
                          env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    out = proc.stdout + proc.stderr
    assert proc.returncode == 0, out[-4000:]
    assert " passed" in proc.stdout and "failed" not in proc.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out
