"""The multi-core CPU baseline program (oracle/su3_cpu_omp.c): it runs on the
host's cores with the paper's constant initialisation, checks that every
output entry is exactly 1+0i, and prints one JSON record; bad arguments are
refused."""

import json
import os
import subprocess

import oracle


def _exe():
    if not os.path.exists(oracle.CPU_OMP):
        oracle.build(force=False)
    return oracle.CPU_OMP


def test_runs_on_several_threads_and_checks_its_result():
    env = dict(os.environ, OMP_NUM_THREADS="3", OMP_PROC_BIND="close", OMP_PLACES="cores")
    proc = subprocess.run([_exe(), "10007", "1", "3", "0"], env=env, capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stderr
    rec = json.loads(proc.stdout)
    assert rec["check_ok"] is True and rec["threads"] == 3 and rec["sites"] == 10007
    assert rec["passes"] >= 3 and rec["sites_per_s"] > 0
    assert abs(rec["gb_s"] - 1152 * rec["sites_per_s"] / 1e9) <= 1e-5 * rec["gb_s"]
    assert rec["omp_proc_bind"] == "close" and rec["omp_places"] == "cores"


def test_bad_arguments_are_refused():
    for args in (["0", "1", "1", "0"], ["-5", "1", "1", "0"], ["100", "1", "0", "0"], ["100"]):
        proc = subprocess.run([_exe(), *args], capture_output=True, text=True, timeout=60)
        assert proc.returncode == 1, args
