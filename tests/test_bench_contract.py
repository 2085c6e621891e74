"""bench.py's command-line contract: one GPU only (N > 1 exits with a
message before anything touches a GPU), and on a GPU one JSON line with the
keys the benchmark record needs."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr and proc.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_hash_ignores_comments_and_layout_only():
    """roofline.traffic is kept only while the kernel code matches the code
    the counters were taken on: comments and whitespace do not count, code
    does."""
    b = _bench_module()
    code = "int f(int x) {\n    return x + 1; // one more\n}\n"
    assert b._code_only(code) == b._code_only("/* header */\nint f(int x)\n{ return x + 1;  }\n")
    assert b._code_only(code) != b._code_only(code.replace("x + 1", "x + 2"))
    assert b._code_only("a /* x\n y */ b // z\nc") == "a b c"
    assert len(b.kernel_source_hash()) == 16


@pytest.mark.gpu
def test_one_json_line_with_the_contract_keys():
    print("[gpu] bench.py short run", flush=True)
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1", "--L",
                           "16", "--bwd-L", "8", "--forms", "f64,soa,soap,copy,shapes,bwd", "--cpu-seconds", "0.5",
                           "--cpu-omp-seconds", "0.5", "--seed", "7"],
                          capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert proc.returncode == 0, proc.stderr[-2000:]
    lines = [l for l in proc.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["unit"] == "sites/s" and "workload" in d["config"]
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 1 and c["value"] > 0 and c["sample"]
    assert c["host"]["nproc"] >= 1 and c["host"]["cpu_model"]
    omp = c["openmp_all_cores"]
    assert omp["check_ok"] is True and omp["threads"] >= 1 and omp["value"] > 0
    assert omp["omp_proc_bind"] == "close" and omp["omp_places"] == "cores"
    assert d["config"]["seed"] == 7
    f = d["forms"]
    assert f["soa"]["vs_site_major"] > 0 and f["soap"]["vs_site_major"] > 0
    assert f["soap"]["pitch"] == (16 ** 4 + 63) // 64 * 64 + 512      # su3_soa_pitch, FP64
    for name in ("soa", "soap"):
        assert f[name]["max_abs_err_vs_oracle"] <= 1e-13
