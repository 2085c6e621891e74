"""Build libsu3.so (the HIP kernels and the C ABI) for gfx950 in-tree.

    python -m paper_2103_00571_amd.build [-D NAME=VALUE ...] [-o OUTPUT]

Compiles every csrc/*.hip file with hipcc into one shared library placed next
to this file, where the Python binding loads it from, and (for the default
output) the C-ABI example program examples/su3_c_api against it.
"""

from __future__ import annotations

import argparse
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsu3.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed FP32 math: keep every FP32 operation a scalar VALU op
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(output: str = LIB, defines: list[str] | None = None, verbose: bool = False,
          extra: list[str] | None = None) -> str:
    """Compile the library; returns the output path. Raises on failure.
    `extra` holds further hipcc flags (the sanitizer test passes host-only
    sanitizer flags here)."""
    cmd = [HIPCC, *FLAGS, *(extra or []), *("-D" + d for d in (defines or [])), *sources(), "-o", output + ".tmp"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 target feature and says
    # so; that line is expected and dropped.
    noise = "is not a recognized feature for this target"
    msgs = [l for l in (proc.stdout + proc.stderr).splitlines() if noise not in l]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s\n%s" % (proc.returncode, " ".join(cmd), "\n".join(msgs)))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(output + ".tmp", output)
    return output


EXAMPLE_SRC = os.path.join(HERE, "examples", "su3_c_api.cpp")
EXAMPLE = os.path.join(HERE, "examples", "su3_c_api")


def build_example(lib: str = LIB, output: str = EXAMPLE) -> str:
    """Compile the C-ABI example program against `lib` (found at run time
    through the rpath, next to this package)."""
    libdir = os.path.dirname(os.path.abspath(lib))
    name = os.path.basename(lib)
    if not (name.startswith("lib") and name.endswith(".so")):
        raise ValueError("library name must be lib<name>.so")
    rpath = "$ORIGIN/" + os.path.relpath(libdir, os.path.dirname(os.path.abspath(output)))
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), EXAMPLE_SRC, "-o", output + ".tmp",
           "-L", libdir, "-l" + name[3:-3], "-Wl,-rpath," + rpath]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s\n%s" % (proc.returncode, " ".join(cmd), proc.stdout + proc.stderr))
    os.replace(output + ".tmp", output)
    return output


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("-D", dest="defines", action="append", default=[], help="extra preprocessor definition")
    ap.add_argument("-o", dest="output", default=LIB)
    args = ap.parse_args()
    print(build(args.output, args.defines, verbose=True))
    if args.output == LIB:
        print(build_example())


if __name__ == "__main__":
    main()
