"""MI355X (gfx950) SU(3) link multiply: HIP kernels behind a C ABI
(include/su3.h, libsu3.so) with a thin PyTorch front end.

    from paper_2103_00571_amd import ops
    c = ops.mult_nn(a, b)          # c[s][j] = a[s][j] @ b[j]

`abi` and `ops` load libsu3.so on first import and raise ImportError when it
is missing or stale; there is no other implementation to fall back to. The
`build` submodule compiles the library and never loads it.
"""

import importlib

__version__ = "0.2.0"

_LAZY = {"abi", "ops"}
_OPS_NAMES = {"SU3_F64", "SU3_F32", "SU3_BF16", "SU3_R12_F32", "SU3_R12C_F32", "SU3_R12_F64", "SU3MultNN",
              "mult_nn", "mult_na", "mult_an", "mat_vec", "mult_nn_autograd", "mult_nn_bwd", "mult_nn_bwd_workspace",
              "mult_nn_soa", "soa_pitch", "aos_to_soa", "soa_to_aos", "pack", "unpack", "stream_copy", "stream_shape",
              "launch_shape", "form_of"}


def __getattr__(name):
    if name in _LAZY:
        return importlib.import_module("." + name, __name__)
    if name in _OPS_NAMES:
        return getattr(importlib.import_module(".ops", __name__), name)
    raise AttributeError("module %r has no attribute %r" % (__name__, name))
