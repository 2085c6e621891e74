"""Benchmark of the SU(3) link multiply c[s][j] = a[s][j] b[j] on one MI355X.

    python bench.py [--steps K | -I K] [--warmup W | -W W] [--L 48] [--seed S] [--forms f64,shard8,soa,...,copy,bwd]

One step is one pass of the product over the whole lattice. The headline is
the FP64 site-major (AoS) product on an L=48 lattice (5,308,416 sites, 3.06 GB
per array): W untimed passes, then K passes timed with HIP events on the
stream the kernel runs on, bracketed by device synchronisation. `value` is
sites per second. The other storage forms, the SoA layout (dense and at the
padded plane pitch su3_soa_pitch gives), one GPU's share of
the lattice split over 8 GPUs (shard8), the L=32 lattice (FP64 and FP32,
site-major and SoA, 100 timed passes), the streaming copy over the same
footprint (the measured bandwidth reference) and the adjoint (L=32) are timed
the same way and reported under "forms", with the streaming ceiling of each
kernel's access shape (su3_stream_shape, "shapes").

Inputs are seeded synthetic Haar SU(3) links (latgen), generated on the host
and copied to HBM before timing starts. A short untimed streaming warm-up
precedes the first timed region. The CPU baseline is the oracle on one pinned
host core (a bounded sample) and, beside it, an OpenMP parallel-for over every
host core. Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SU(3) link-mult sites/s & % HBM peak, L=48 FP64 vs FP32/recon-12"
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
FLOP_PER_SITE = 864            # paper's count: 4 x 27 x (4 mul + 4 add)
MATVEC_FLOP_PER_SITE = 4 * 3 * 3 * 8   # 4 links x 3 rows x 3 complex multiply-adds of 8 flop
# algorithmic bytes per site: a read once + c written once (b ignored)
BYTES_PER_SITE = {"f64": 1152, "soa": 1152, "soap": 1152, "f32": 576, "bf16": 288, "r12": 480,
                  "r12c": 384, "r12f64": 960, "na": 1152, "an": 1152, "matvec": 816,
                  "soa32": 576, "soap32": 576, "na32": 576, "an32": 576, "matvec32": 408}
BWD_BYTES_PER_SITE = {"f64": 3 * 576, "f32": 3 * 288}   # a, dC read; dA written
# The paper's own figures for this kernel, on its hardware (context, not a
# target): 864 flop per site, sites/s = GF/s * 1e9 / 864.
PAPER_CONTEXT = {
    "xeon_2x_clx8280_56c_fp32_L32_best": {"gflop_s": 193.54, "gb_s_padded_site": 143.46, "sites_per_s": 2.24e8,
                                          "where": "section Performance on Xeon (empty constructors, parallel first touch)"},
    "xeon_2x_clx8280_56c_fp32_L32_openmp_v1": {"gflop_s": 94.82, "sites_per_s": 1.10e8,
                                               "where": "section Performance on Xeon (OpenMP versions table, Version 1, 200 iterations)"},
    "piuma_32_cores_fp64_L32": {"gb_s": 108.0, "vs_32_clx_cores": 1.48,
                                "where": "section Optimization on PIUMA (simulator)"},
    "piuma_16_cores_fp64_L32": {"gflop_s": 43.88, "gb_s": 61.42, "sites_per_s": 5.08e7,
                                "where": "section Optimization on PIUMA (simulator)"},
}
KERNEL_SOURCES = ["paper_2103_00571_amd/csrc/su3_fwd.hip", "paper_2103_00571_amd/csrc/su3_internal.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fwd_aos_f64_L48.json")
# Untimed warm-up, in seconds, of every leg after the headline (which runs W
# untimed steps right after the device warm-up).
LEG_WARM_S = 0.1


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """The C++ source with comments removed and whitespace runs collapsed, so
    that an edit of comments or layout does not count as a kernel change."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def time_launches(fn, steps: int, warmup: int, torch, warm_seconds: float = 0.0) -> float:
    """Average milliseconds per call of fn() over `steps` back-to-back calls,
    from HIP events on the current stream (where fn launches). Before timing:
    `warmup` untimed calls, then more untimed calls until at least
    `warm_seconds` of them have run (the GPU takes tens of milliseconds to
    return to its steady rate after an idle stretch, such as host-side input
    generation between two legs)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if warm_seconds > 0:
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < warm_seconds:
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def traffic_record():
    """HBM bytes per launch of the FP64 AoS kernel at L=48 from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by what
    it reads for the streaming copy of known size), or None if the summary is
    missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def host_info() -> dict:
    """CPU model, core counts and NUMA node count of the host."""
    info = {"cpu_model": "unknown", "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(),
            "numa_nodes": None, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key == "Model name":
                info["cpu_model"] = val
            elif key in ("Socket(s)", "Core(s) per socket", "Thread(s) per core", "NUMA node(s)"):
                info[key.lower().replace("(s)", "s").replace(" ", "_")] = int(val) if val.isdigit() else val
    except (OSError, subprocess.SubprocessError):
        pass
    if info["cpu_model"] == "unknown":
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["cpu_model"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        info["numa_nodes"] = len([d for d in os.listdir("/sys/devices/system/node") if re.fullmatch(r"node\d+", d)])
    except OSError:
        pass
    return info


def cpu_baseline_leg(a, b, sample_idx, seconds: float, L: int):
    """The oracle (plain single-threaded C, FP64) timed on one host core on
    a bounded sample of the same workload -- the first 2^20 sites of the
    lattice, which are exactly the L=32 lattice of the same seed -- and its
    reference values on the sampled sites used for the error report."""
    import numpy as np

    import oracle
    O = oracle.default()
    sample = np.ascontiguousarray(a[: 1 << 20])
    O.mult_nn(sample[:1024], b)            # load and warm
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    # pin this thread (the one that calls the oracle) to one core for the
    # timing, then give it back its cores
    os.sched_setaffinity(0, {core})
    try:
        passes, t0 = 0, time.perf_counter()
        while True:
            O.mult_nn(sample, b)
            passes += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    finally:
        os.sched_setaffinity(0, allowed)
    rate = passes * sample.shape[0] / el
    ref = O.mult_nn(a[sample_idx], b)
    rec = {"value": rate, "unit": "sites/s", "cores": 1, "kind": "oracle",
           "sample": "first %d sites of the L=%d lattice (the L=32 lattice of the same seed), FP64 AoS, "
                     "%d passes in %.1f s, single thread pinned to CPU %d" % (sample.shape[0], L, passes, el, core),
           "gb_s": rate * 1152 / 1e9, "pinned_cpu": core, "host": host_info()}
    return rec, ref, O


def cpu_omp_leg(sites: int, seconds: float) -> dict:
    """The multi-core CPU baseline: the product over `sites` sites on every
    host core the process may use, one OpenMP parallel-for over sites with
    parallel first-touch initialisation and close thread binding (the paper's
    best Xeon setup), run as a child process. Returns its JSON record."""
    import oracle
    if not os.path.exists(oracle.CPU_OMP):
        oracle.build(force=False)
    env = dict(os.environ, OMP_PROC_BIND="close", OMP_PLACES="cores")
    cmd = [oracle.CPU_OMP, str(sites), "2", "5", "%.1f" % seconds]
    proc = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if proc.returncode != 0:
        return {"error": "exit %d: %s" % (proc.returncode, (proc.stdout + proc.stderr)[-500:])}
    rec = json.loads(proc.stdout.strip().splitlines()[-1])
    rec.update({"unit": "sites/s", "value": rec["sites_per_s"], "cores": rec["threads"],
                "kind": "openmp parallel-for, all host cores (not the oracle)",
                "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
                "sample": "the full %d-site lattice, FP64 AoS, paper's constant initialisation, parallel first touch"
                          % sites})
    return rec


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # -I and -W are SU3_Bench's own names for the timed and warm-up iterations
    ap.add_argument("--steps", "-I", type=int, default=100)
    ap.add_argument("--warmup", "-W", type=int, default=20)
    ap.add_argument("--L", type=int, default=48)
    ap.add_argument("--bwd-L", type=int, default=32)
    ap.add_argument("--seed", type=int, default=1,
                    help="seed of a; b, dC and the colour vectors take seed+1, seed+2, seed+3")
    ap.add_argument("--forms",
                    default="f64,shard8,l32,soa,soap,f32,bf16,r12,r12c,r12f64,na,an,matvec,fp32more,setup,copy,shapes,bwd")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-omp", action="store_true", help="skip the multi-core OpenMP CPU baseline")
    ap.add_argument("--cpu-omp-seconds", type=float, default=4.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU kernel "
              "(sites shard across GPUs with no communication in the forward pass); use --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import latgen
    from paper_2103_00571_amd import ops

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    forms = [f for f in args.forms.split(",") if f]
    L = args.L
    sites = L ** 4

    t0 = time.perf_counter()
    a = latgen.random_lattice(sites, seed=args.seed)
    b = latgen.random_b(seed=args.seed + 1)
    log("generated L=%d lattice (%d sites, %.2f GB) in %.1f s" % (L, sites, a.nbytes / 1e9, time.perf_counter() - t0))
    ta = torch.from_numpy(a).to(dev)
    tb64 = torch.from_numpy(b).to(dev)
    tb32 = tb64.to(torch.complex64)
    torch.cuda.synchronize()

    results = {}
    outputs = {}

    def record(name, ms, nbytes_site, n_sites):
        gbs = nbytes_site * n_sites / (ms * 1e-3) / 1e9
        flop = MATVEC_FLOP_PER_SITE if name.startswith("matvec") else FLOP_PER_SITE
        results[name] = {"ms": ms, "sites_per_s": n_sites / (ms * 1e-3), "gb_s": gbs,
                         "frac_hbm_peak": gbs / HBM_PEAK_GBS, "gflop_s": flop * n_sites / (ms * 1e-3) / 1e9}
        log("%-5s %8.4f ms  %.3e sites/s  %7.1f GB/s  (%.1f%% of 8 TB/s)"
            % (name, ms, n_sites / (ms * 1e-3), gbs, 100 * gbs / HBM_PEAK_GBS))

    # ---- device warm-up (untimed) --------------------------------------------
    # About 0.2 s of the streaming copy over the headline's footprint, so that
    # clocks and memory are in their steady state before the first timed
    # region; the first dispatches on a cold device run several percent slow.
    c64 = torch.empty_like(ta)
    t0w, nw = time.perf_counter(), 0
    while time.perf_counter() - t0w < 0.2:
        for _ in range(10):
            ops.stream_copy(ta, c64)
        torch.cuda.synchronize()
        nw += 10
    log("device warm-up: %d streaming copies in %.2f s" % (nw, time.perf_counter() - t0w))

    # ---- headline: FP64 AoS ------------------------------------------------
    grid, block = ops.launch_shape(sites, ops.SU3_F64)
    ms64 = time_launches(lambda: ops.mult_nn(ta, tb64, out=c64), args.steps, args.warmup, torch)
    record("f64", ms64, BYTES_PER_SITE["f64"], sites)
    outputs["f64"] = c64

    # ---- one GPU's share when the lattice is split over 8 GPUs ----------------
    # (sites are independent and b is replicated, so a shard is the same kernel
    # on a contiguous range of sites)
    if "shard8" in forms and sites >= 8:
        ns = sites // 8
        xs, ys = ta[:ns], torch.empty_like(ta[:ns])
        ms = time_launches(lambda: ops.mult_nn(xs, tb64, out=ys), args.steps, args.warmup, torch, LEG_WARM_S)
        record("shard8", ms, BYTES_PER_SITE["f64"], ns)
        results["shard8"]["sites"] = ns
        del ys

    # ---- the L=32 lattice (1,048,576 sites): 100 timed passes ----------------
    # The first 2^20 sites of the lattice are the L=32 lattice of the same seed
    # (entries are a function of the site index only). Site-major FP64 and
    # FP32 and the SoA layout in both, each into a preallocated output.
    n32 = 32 ** 4
    steps32 = max(args.steps, 100)
    if "l32" in forms and sites >= n32:
        x64 = ta[:n32]
        y64 = torch.empty_like(x64)
        ms = time_launches(lambda: ops.mult_nn(x64, tb64, out=y64), steps32, args.warmup, torch, LEG_WARM_S)
        record("f64_L32", ms, BYTES_PER_SITE["f64"], n32)
        results["f64_L32"].update({"sites": n32, "steps": steps32})
        x32 = ops.pack(x64, ops.SU3_F32)
        y32 = torch.empty_like(x32)
        ms = time_launches(lambda: ops.mult_nn(x32, tb32, out=y32), steps32, args.warmup, torch, LEG_WARM_S)
        record("f32_L32", ms, BYTES_PER_SITE["f32"], n32)
        results["f32_L32"].update({"sites": n32, "steps": steps32})
        for name, x, tb, key in (("soa_L32", x64, tb64, "f64_L32"), ("soa32_L32", x32, tb32, "f32_L32")):
            sa = ops.aos_to_soa(x)
            sc = torch.empty_like(sa)
            ms = time_launches(lambda: ops.mult_nn_soa(sa, tb, out=sc), steps32, args.warmup, torch, LEG_WARM_S)
            record(name, ms, BYTES_PER_SITE["soa" if name == "soa_L32" else "soa32"], n32)
            results[name].update({"sites": n32, "steps": steps32,
                                  "vs_site_major": results[key]["ms"] / ms})
            del sa, sc
        if "soap" in forms:
            # the padded SoA layout at the pitch su3_soa_pitch recommends
            for name, x, tb, key, form in (("soap_L32", x64, tb64, "f64_L32", ops.SU3_F64),
                                           ("soap32_L32", x32, tb32, "f32_L32", ops.SU3_F32)):
                pitch = ops.soa_pitch(n32, form)
                sa = ops.aos_to_soa(x, pitch)
                sc = torch.empty_like(sa)
                ms = time_launches(lambda: ops.mult_nn_soa(sa, tb, out=sc, sites=n32), steps32, args.warmup, torch,
                                   LEG_WARM_S)
                record(name, ms, BYTES_PER_SITE["soap" if form == ops.SU3_F64 else "soap32"], n32)
                results[name].update({"sites": n32, "steps": steps32, "pitch": pitch,
                                      "vs_site_major": results[key]["ms"] / ms})
                del sa, sc
        del y64, x32, y32

    # ---- streaming copy over the same footprint (measured bandwidth) -------
    if "copy" in forms:
        dst = torch.empty_like(ta)
        msc = time_launches(lambda: ops.stream_copy(ta, dst), args.steps, args.warmup, torch, LEG_WARM_S)
        msd = time_launches(lambda: dst.copy_(ta), max(10, args.steps // 4), 2, torch, LEG_WARM_S)
        nb = 2 * a.nbytes
        results["copy"] = {"ms": msc, "gb_s": nb / (msc * 1e-3) / 1e9, "bytes_moved": nb,
                           "torch_copy_ms": msd, "torch_copy_gb_s": nb / (msd * 1e-3) / 1e9}
        log("copy  %8.4f ms  %7.1f GB/s (library kernel); torch copy_ %7.1f GB/s"
            % (msc, nb / (msc * 1e-3) / 1e9, nb / (msd * 1e-3) / 1e9))
        del dst

    # ---- ceilings of the kernels' access shapes (su3_stream_shape) ----------
    # Each shape streams the footprint of the kernel it stands beside with no
    # arithmetic; the best rate over a sweep of the occupancy cap is that
    # shape's streaming ceiling on this GPU.
    if "shapes" in forms:
        bsites = args.bwd_L ** 4
        # (shape, tiles, tile order of the kernels beside it, kernels)
        shapes = [((3, 0, 3), 12 * sites // 64, 1, "f64, f32, bf16, r12c, na"),
                  ((3, 0, 3), 12 * sites // 64, 0, "none (the same shape with tile = workgroup index)"),
                  ((1, 0, 1), 36 * sites // 64, 0, "copy"),
                  ((3, 3, 3), 12 * bsites // 64, 0, "bwd_f64, bwd_f32"),
                  ((6, 0, 9), 2 * sites // 64, 1, "r12, r12f64"),
                  ((9, 0, 9), 4 * sites // 64, 1, "an")]
        abytes = ta.view(torch.uint8).reshape(-1)
        bbytes = c64.view(torch.uint8).reshape(-1)
        cbytes = torch.empty(max(t * 1024 * sh[2] for sh, t, _, _ in shapes), dtype=torch.uint8, device=dev)
        res = {}
        for (ia, ib, io), tiles, order, beside in shapes:
            if tiles * 1024 * max(ia, ib) > abytes.numel():
                continue
            A, C = abytes[: tiles * 1024 * ia], cbytes[: tiles * 1024 * io]
            B = bbytes[: tiles * 1024 * ib] if ib else None
            nbytes = (ia + ib + io) * tiles * 1024
            best = None
            for cap in (0, 32, 24, 16, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4):
                ms = time_launches(lambda: ops.stream_shape(A, B, C, ia, ib, io, cap, order), 20, 3, torch)
                gbs = nbytes / (ms * 1e-3) / 1e9
                if best is None or gbs > best[0]:
                    best = (gbs, cap, ms)
            key = "%d+%d in, %d out" % (ia, ib, io)
            if key in res:
                key += ", %s order" % ("xcd" if order else "index")
            res[key] = {"gb_s": best[0], "waves_per_cu": best[1], "ms": best[2], "bytes": nbytes,
                        "tile_order": "xcd" if order else "index", "kernels": beside}
            log("shape %-14s ceiling %7.1f GB/s (cap %d, %s order)  beside %s"
                % (key, best[0], best[1], "xcd" if order else "index", beside))
        results["shapes"] = res
        del cbytes

    # ---- SoA ---------------------------------------------------------------
    if "soa" in forms:
        sa = ops.aos_to_soa(ta)
        sc = torch.empty_like(sa)
        ms = time_launches(lambda: ops.mult_nn_soa(sa, tb64, out=sc), args.steps, args.warmup, torch, LEG_WARM_S)
        record("soa", ms, BYTES_PER_SITE["soa"], sites)
        results["soa"]["vs_site_major"] = ms64 / ms
        outputs["soa"] = ops.soa_to_aos(sc)
        del sa, sc
    if "soap" in forms:
        pitch = ops.soa_pitch(sites, ops.SU3_F64)
        sa = ops.aos_to_soa(ta, pitch)
        sc = torch.empty_like(sa)
        ms = time_launches(lambda: ops.mult_nn_soa(sa, tb64, out=sc, sites=sites), args.steps, args.warmup, torch,
                           LEG_WARM_S)
        record("soap", ms, BYTES_PER_SITE["soap"], sites)
        results["soap"].update({"pitch": pitch, "vs_site_major": ms64 / ms})
        outputs["soap"] = ops.soa_to_aos(sc, sites)
        del sa, sc

    # ---- reduced storage forms -----------------------------------------------
    for name, code in (("f32", ops.SU3_F32), ("bf16", ops.SU3_BF16), ("r12", ops.SU3_R12_F32)):
        if name not in forms:
            continue
        x = ops.pack(ta, code)
        y = ops.mult_nn(x, tb32)
        ms = time_launches(lambda: ops.mult_nn(x, tb32, out=y), args.steps, args.warmup, torch, LEG_WARM_S)
        record(name, ms, BYTES_PER_SITE[name], sites)
        outputs[name] = y
        del x
    # ---- compressed-output and FP64 reconstruct-12 -------------------------
    if "r12c" in forms:
        x = ops.pack(ta, ops.SU3_R12C_F32)
        y = ops.mult_nn(x, tb32, form=ops.SU3_R12C_F32)
        ms = time_launches(lambda: ops.mult_nn(x, tb32, out=y, form=ops.SU3_R12C_F32), args.steps, args.warmup,
                           torch, LEG_WARM_S)
        record("r12c", ms, BYTES_PER_SITE["r12c"], sites)
        outputs["r12c"] = ops.unpack(y, ops.SU3_R12C_F32)   # product with row 2 rebuilt, for the error report
        del x, y
    if "r12f64" in forms:
        x = ops.pack(ta, ops.SU3_R12_F64)
        y = ops.mult_nn(x, tb64)
        ms = time_launches(lambda: ops.mult_nn(x, tb64, out=y), args.steps, args.warmup, torch, LEG_WARM_S)
        record("r12f64", ms, BYTES_PER_SITE["r12f64"], sites)
        outputs["r12f64"] = y
        del x
    # ---- the other products (FP64): a b^H, a^H b, matrix x colour vector -------
    for name, fn in (("na", ops.mult_na), ("an", ops.mult_an)):
        if name in forms:
            y = torch.empty_like(ta)
            ms = time_launches(lambda: fn(ta, tb64, out=y), args.steps, args.warmup, torch, LEG_WARM_S)
            record(name, ms, BYTES_PER_SITE[name], sites)
            del y
    if "matvec" in forms:
        tv = torch.from_numpy(latgen.complex_normal_lattice(sites, seed=args.seed + 3)[:, 0, 0, :].copy()).to(dev)
        w = ops.mat_vec(ta, tv)
        ms = time_launches(lambda: ops.mat_vec(ta, tv, out=w), args.steps, args.warmup, torch, LEG_WARM_S)
        record("matvec", ms, BYTES_PER_SITE["matvec"], sites)
        del tv, w
    # ---- setup kernels: layout transforms and storage-form conversions -------
    # (off the product's timed path; bytes = source read + destination written)
    if "setup" in forms:
        t0s = time.perf_counter()
        k = max(10, args.steps // 5)
        sa = ops.aos_to_soa(ta)
        back = ops.soa_to_aos(sa)
        setup = {}

        def rec_setup(name, fn, nbytes):
            ms = time_launches(fn, k, 3, torch, LEG_WARM_S)
            setup[name] = {"ms": ms, "gb_s": nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes}
            log("setup %-12s %8.4f ms  %7.1f GB/s" % (name, ms, nbytes / (ms * 1e-3) / 1e9))

        rec_setup("aos_to_soa", lambda: ops.aos_to_soa(ta), 1152 * sites)
        rec_setup("soa_to_aos", lambda: ops.soa_to_aos(sa), 1152 * sites)
        del sa, back
        for name, code, packed in (("f32", ops.SU3_F32, 288), ("bf16", ops.SU3_BF16, 144),
                                   ("r12", ops.SU3_R12_F32, 192), ("r12f64", ops.SU3_R12_F64, 384)):
            x = ops.pack(ta, code)
            rec_setup("pack_" + name, lambda: ops.pack(ta, code), (576 + packed) * sites)
            rec_setup("unpack_" + name, lambda: ops.unpack(x), (packed + 576) * sites)
            del x
        results["setup"] = setup
        log("setup leg %.1f s" % (time.perf_counter() - t0s))

    # ---- FP32 variants of the SoA product and the other products ------------
    if "fp32more" in forms:
        t32 = ta.to(torch.complex64)
        sa = ops.aos_to_soa(t32)
        sc = torch.empty_like(sa)
        record("soa32", time_launches(lambda: ops.mult_nn_soa(sa, tb32, out=sc), args.steps, args.warmup, torch, LEG_WARM_S),
               BYTES_PER_SITE["soa32"], sites)
        if "f32" in results:
            results["soa32"]["vs_site_major"] = results["f32"]["ms"] / results["soa32"]["ms"]
        del sa, sc
        if "soap" in forms:
            pitch = ops.soa_pitch(sites, ops.SU3_F32)
            sa = ops.aos_to_soa(t32, pitch)
            sc = torch.empty_like(sa)
            record("soap32", time_launches(lambda: ops.mult_nn_soa(sa, tb32, out=sc, sites=sites), args.steps,
                                           args.warmup, torch, LEG_WARM_S), BYTES_PER_SITE["soap32"], sites)
            results["soap32"]["pitch"] = pitch
            if "f32" in results:
                results["soap32"]["vs_site_major"] = results["f32"]["ms"] / results["soap32"]["ms"]
            del sa, sc
        y = torch.empty_like(t32)
        for name, fn in (("na32", ops.mult_na), ("an32", ops.mult_an)):
            record(name, time_launches(lambda: fn(t32, tb32, out=y), args.steps, args.warmup, torch, LEG_WARM_S),
                   BYTES_PER_SITE[name], sites)
        del y
        tv = torch.from_numpy(latgen.complex_normal_lattice(sites, seed=args.seed + 3)[:, 0, 0, :].copy()).to(dev)
        tv = tv.to(torch.complex64)
        w = ops.mat_vec(t32, tv)
        record("matvec32", time_launches(lambda: ops.mat_vec(t32, tv, out=w), args.steps, args.warmup, torch, LEG_WARM_S),
               BYTES_PER_SITE["matvec32"], sites)
        del t32, tv, w
    for name in ("f32", "bf16", "r12", "r12c", "r12f64", "soa", "soap"):
        if name in results:
            results[name]["speedup_vs_f64"] = ms64 / results[name]["ms"]
    # the paper counts a read and c written as its padded Site struct, 640 B
    # (FP64) or 320 B (FP32) each, and ignores b (section Background)
    for name, padded in (("f64", 1280), ("f32", 640)):
        if name in results:
            results[name]["gb_s_paper_convention"] = padded * results[name]["sites_per_s"] / 1e9
    if "copy" in results:
        for name, r in results.items():
            if name not in ("copy", "shapes", "setup") and "gb_s" in r:
                r["frac_of_measured_copy"] = r["gb_s"] / results["copy"]["gb_s"]

    # ---- adjoint (L = bwd-L) -----------------------------------------------
    if "bwd" in forms:
        bs = args.bwd_L ** 4
        xa = torch.from_numpy(np.ascontiguousarray(a[:bs])).to(dev) if bs <= sites else None
        if xa is not None:
            xdc = torch.from_numpy(latgen.complex_normal_lattice(bs, seed=args.seed + 2)).to(dev)
            for name, dt, tb in (("bwd_f64", torch.complex128, tb64), ("bwd_f32", torch.complex64, tb32)):
                xa_, xdc_ = xa.to(dt), xdc.to(dt)
                # preallocated outputs and workspace, as in the forward legs
                da_, db_ = torch.empty_like(xa_), torch.empty((4, 3, 3), dtype=torch.complex128, device=dev)
                ws_ = ops.mult_nn_bwd_workspace(bs, ops.form_of(xa_), dev)
                ms = time_launches(lambda: ops.mult_nn_bwd(xa_, tb, xdc_, da=da_, db=db_, ws=ws_), args.steps,
                                   args.warmup, torch, LEG_WARM_S)
                nb = BWD_BYTES_PER_SITE[name[4:]] * bs
                results[name] = {"ms": ms, "sites_per_s": bs / (ms * 1e-3), "gb_s": nb / (ms * 1e-3) / 1e9,
                                 "frac_hbm_peak": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "L": args.bwd_L,
                                 "workspace_bytes": ws_.numel()}
                del da_, db_, ws_
                log("%-7s %8.4f ms  %.3e sites/s  %7.1f GB/s" % (name, ms, bs / (ms * 1e-3), nb / (ms * 1e-3) / 1e9))
            del xa, xdc

    # ---- CPU baseline (oracle) and error report on sampled sites -------------
    cpu = None
    if not args.no_cpu_baseline:
        idx = np.unique(np.concatenate([np.random.default_rng(48).choice(sites, min(4096, sites), replace=False),
                                        [0, sites - 1]]))
        cpu, ref, O = cpu_baseline_leg(a, b, idx, args.cpu_seconds, L)
        log("oracle on host: %.3e sites/s (%s)" % (cpu["value"], cpu["sample"]))
        if "f64_L32" in results:
            # the oracle ran on exactly the L=32 lattice the GPU leg timed
            results["f64_L32"]["oracle_sites_per_s"] = cpu["value"]
            results["f64_L32"]["speedup_vs_oracle"] = results["f64_L32"]["sites_per_s"] / cpu["value"]
        if not args.no_cpu_omp:
            omp = cpu_omp_leg(sites, args.cpu_omp_seconds)
            cpu["openmp_all_cores"] = omp
            if "value" in omp:
                log("openmp on %d host threads: %.3e sites/s, %.1f GB/s" % (omp["threads"], omp["value"],
                                                                           omp["gb_s"]))
            else:
                log("openmp baseline failed: %s" % omp.get("error"))
        tidx = torch.from_numpy(idx).to(dev)
        for name, out in outputs.items():
            if name == "bf16":
                got = O.widen_bf16(out[tidx].view(torch.int16).cpu().numpy().view(np.uint16))
            else:
                got = out[tidx].cpu().numpy().astype(np.complex128)
            results[name]["max_abs_err_vs_oracle"] = O.max_abs_diff(got, ref)
            results[name]["unitarity_dev"] = O.unitarity_dev(got)
            results[name]["err_sample_sites"] = int(idx.size)

    # ---- roofline of the dominant kernel ---------------------------------------
    alg_bytes = BYTES_PER_SITE["f64"] * sites
    achieved = alg_bytes / (ms64 * 1e-3) / 1e9
    traffic = traffic_record() if L == 48 else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_over_algorithmic": None if traffic is None else traffic / alg_bytes,
                "kernel": "su3::fwd_aos<FormF64>", "algorithmic_bytes_per_launch": alg_bytes,
                "bytes_per_site": BYTES_PER_SITE["f64"], "grid": grid, "block": block}
    if "copy" in results:
        roofline["frac_of_measured_copy"] = achieved / results["copy"]["gb_s"]
    if "shapes" in results and "3+0 in, 3 out" in results["shapes"]:
        ceil = results["shapes"]["3+0 in, 3 out"]["gb_s"]
        roofline["shape_ceiling_gb_s"] = ceil
        roofline["frac_of_shape_ceiling"] = achieved / ceil

    line = {
        "metric": METRIC,
        "value": results["f64"]["sites_per_s"],
        "unit": "sites/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Haar SU(3) links, SplitMix64 + Box-Muller)",
        "config": {"workload": "su3_mult_nn FP64 AoS, L=%d (%d sites, 4 links/site)" % (L, sites),
                   "L": L, "sites": sites, "layout": "aos", "precision": "f64",
                   "bytes_per_site": BYTES_PER_SITE["f64"], "flop_per_site": FLOP_PER_SITE, "seed": args.seed},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": results,
        "paper_context": PAPER_CONTEXT,
        "device": torch.cuda.get_device_name(dev),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
