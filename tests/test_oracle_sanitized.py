"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

`oracle/su3_oracle.c` is compiled again with -fsanitize=address,undefined
(host code only: the oracle has no GPU code) into a temporary library, and
every pin of the oracle runs against that build in a child Python process
with the ASan runtime preloaded, so that numpy's buffers carry redzones and
any read or write past an array the oracle is handed, any use of freed
memory and any undefined arithmetic (signed overflow, bad shifts, misaligned
access) stops the run with a report.

The multi-core baseline program (`oracle/su3_cpu_omp.c`) is built with the
same sanitizers and run once on a small lattice.
"""

import os
import subprocess
import sys
import textwrap

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _env():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's ASan runtime is not installed")
    env = dict(os.environ)
    # ASan must come first among preloaded libraries; anything already
    # preloaded stays in the list after it
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = os.pathsep.join([ROOT, HERE] + ([env["PYTHONPATH"]] if env.get("PYTHONPATH") else []))
    return env


def test_oracle_pins_under_sanitizers(tmp_path):
    so = tmp_path / "liboracle_san.so"
    cflags = [f for f in oracle.CFLAGS if f != "-O2"] + ["-O1"]
    subprocess.run(["gcc", *cflags, *SAN_FLAGS, os.path.join(ROOT, "oracle", "su3_oracle.c"), "-o", str(so), "-lm"],
                   check=True)
    script = tmp_path / "run_pins.py"
    script.write_text(textwrap.dedent("""
        import importlib.util, inspect, os, sys
        import oracle
        here = %r
        O = oracle.Oracle(oracle.load(%r))
        ran = 0
        for fname in ("test_oracle_pins.py", "test_oracle_next.py", "test_oracle_exact.py"):
            spec = importlib.util.spec_from_file_location(fname[:-3], os.path.join(here, fname))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            for name, f in sorted(vars(mod).items()):
                if name.startswith("test_") and "O" in inspect.signature(f).parameters:
                    f(O)
                    ran += 1
        print("pins passed under sanitizers:", ran)
    """ % (HERE, str(so))))
    proc = subprocess.run([sys.executable, str(script)], env=_env(), capture_output=True, text=True, timeout=900)
    assert proc.returncode == 0, (proc.stdout + proc.stderr)[-4000:]
    assert "pins passed under sanitizers:" in proc.stdout
    assert int(proc.stdout.split(":")[-1]) >= 30
    assert "runtime error" not in proc.stderr and "AddressSanitizer" not in proc.stderr


def test_cpu_baseline_program_under_sanitizers(tmp_path):
    exe = tmp_path / "su3_cpu_omp_san"
    subprocess.run(["gcc", *oracle.OMP_CFLAGS, *SAN_FLAGS, os.path.join(ROOT, "oracle", "su3_cpu_omp.c"), "-o",
                    str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               OMP_NUM_THREADS="4")
    proc = subprocess.run([str(exe), "4099", "1", "2", "0"], env=env, capture_output=True, text=True, timeout=300)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert '"check_ok": true' in proc.stdout


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    """The check above can fail: a copy of the oracle whose forward loop runs
    one site past the end is reported as a heap-buffer-overflow."""
    src = open(os.path.join(ROOT, "oracle", "su3_oracle.c")).read()
    start = src.index("void su3o_mult_nn(")
    loop = "for (int64_t i = 0; i < sites; ++i)"
    at = src.index(loop, start)
    c_path, so = tmp_path / "overflow.c", tmp_path / "liboverflow.so"
    c_path.write_text(src[:at] + loop.replace("<", "<=") + src[at + len(loop):])
    cflags = [f for f in oracle.CFLAGS if f != "-O2"] + ["-O1"]
    subprocess.run(["gcc", *cflags, *SAN_FLAGS, str(c_path), "-o", str(so), "-lm"], check=True)
    script = tmp_path / "run.py"
    script.write_text(textwrap.dedent("""
        import latgen, oracle
        O = oracle.Oracle(oracle.load(%r))
        O.mult_nn(latgen.random_lattice(100, seed=1), latgen.random_b(seed=2))
        print("no report")
    """ % str(so)))
    proc = subprocess.run([sys.executable, str(script)], env=_env(), capture_output=True, text=True, timeout=300)
    assert proc.returncode != 0 and "heap-buffer-overflow" in proc.stderr
