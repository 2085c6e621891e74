"""ctypes binding of libsu3.so: the entry points of include/su3.h under the
same names, taking device pointers and stream handles as Python ints.

Nothing here computes: every function marshals its arguments and calls the
HIP library. If the library is not built this module raises on import, so no
caller can silently fall back to another implementation.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SU3_LIB_PATH selects another build of the same library (a sanitized one in
# the tests); by default the in-tree libsu3.so.
LIB_PATH = os.environ.get("SU3_LIB_PATH") or os.path.join(_HERE, "libsu3.so")

# su3.h constants
ABI_VERSION = 6
SU3_F64, SU3_F32, SU3_BF16, SU3_R12_F32, SU3_R12C_F32, SU3_R12_F64 = 0, 1, 2, 3, 4, 5
SU3_OK = 0
SU3_ERR_NULL, SU3_ERR_SIZE, SU3_ERR_ALIGN, SU3_ERR_PRECISION = -1, -2, -3, -4
SU3_ERR_OVERLAP, SU3_ERR_WORKSPACE, SU3_ERR_HIP = -5, -6, -7
SU3_BWD_SCRATCH_BYTES = 64 << 20   # workspace of su3_mult_nn_bwd_noalloc

# every symbol su3.h declares, with (argtypes, restype)
_P, _I64, _I, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
SIGNATURES = {
    "su3_abi_version": ([], _I),
    "su3_status_string": ([_I], ctypes.c_char_p),
    "su3_mult_nn": ([_P, _P, _P, _I64, _I, _P], _I),
    "su3_mult_nn_soa": ([_P, _P, _P, _I64, _I, _P], _I),
    "su3_mult_na": ([_P, _P, _P, _I64, _I, _P], _I),
    "su3_mult_an": ([_P, _P, _P, _I64, _I, _P], _I),
    "su3_mat_vec": ([_P, _P, _P, _I64, _I, _P], _I),
    "su3_aos_to_soa": ([_P, _P, _I64, _I, _P], _I),
    "su3_soa_to_aos": ([_P, _P, _I64, _I, _P], _I),
    "su3_mult_nn_soa_pitched": ([_P, _P, _P, _I64, _I64, _I, _P], _I),
    "su3_soa_pitch": ([_I64, _I, ctypes.POINTER(ctypes.c_int64)], _I),
    "su3_aos_to_soa_pitched": ([_P, _P, _I64, _I64, _I, _P], _I),
    "su3_soa_to_aos_pitched": ([_P, _P, _I64, _I64, _I, _P], _I),
    "su3_pack": ([_P, _P, _I64, _I, _P], _I),
    "su3_unpack": ([_P, _P, _I64, _I, _P], _I),
    "su3_mult_nn_bwd_workspace_bytes": ([_I64, _I], _SZ),
    "su3_mult_nn_bwd": ([_P, _P, _P, _P, _P, _I64, _I, _P, _SZ, _P], _I),
    "su3_mult_nn_bwd_noalloc": ([_P, _P, _P, _P, _P, _I64, _I, _P], _I),
    "su3_stream_copy": ([_P, _P, _I64, _P], _I),
    "su3_stream_shape": ([_P, _P, _P, _I64, _I, _I, _I, _I, _I, _P], _I),
    "su3_launch_shape": ([_I64, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)], _I),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libsu3.so is not built (%s); run `python -m paper_2103_00571_amd.build` "
            "from the repository root" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    v = lib.su3_abi_version()
    if v != ABI_VERSION:
        raise ImportError("libsu3.so ABI version %d, binding expects %d: rebuild" % (v, ABI_VERSION))
    return lib


lib = _load()


class SU3Error(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s" % (where, status_string(status)))


def status_string(status: int) -> str:
    return lib.su3_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != SU3_OK:
        raise SU3Error(status, where)


# ---- entry points, same names and argument order as su3.h ------------------

def su3_abi_version() -> int:
    return lib.su3_abi_version()


def su3_status_string(status: int) -> str:
    return status_string(status)


def su3_mult_nn(a: int, b: int, c: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_mult_nn(a, b, c, sites, precision, stream)


def su3_mult_na(a: int, b: int, c: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_mult_na(a, b, c, sites, precision, stream)


def su3_mult_an(a: int, b: int, c: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_mult_an(a, b, c, sites, precision, stream)


def su3_mat_vec(a: int, v: int, w: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_mat_vec(a, v, w, sites, precision, stream)


def su3_mult_nn_soa(a: int, b: int, c: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_mult_nn_soa(a, b, c, sites, precision, stream)


def su3_aos_to_soa(src: int, dst: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_aos_to_soa(src, dst, sites, precision, stream)


def su3_soa_to_aos(src: int, dst: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_soa_to_aos(src, dst, sites, precision, stream)


def su3_mult_nn_soa_pitched(a: int, b: int, c: int, sites: int, pitch: int, precision: int, stream: int) -> int:
    return lib.su3_mult_nn_soa_pitched(a, b, c, sites, pitch, precision, stream)


def su3_soa_pitch(sites: int, precision: int) -> int:
    """The recommended plane pitch; raises SU3Error on a bad argument."""
    p = ctypes.c_int64()
    check(lib.su3_soa_pitch(sites, precision, ctypes.byref(p)), "su3_soa_pitch")
    return p.value


def su3_aos_to_soa_pitched(src: int, dst: int, sites: int, pitch: int, precision: int, stream: int) -> int:
    return lib.su3_aos_to_soa_pitched(src, dst, sites, pitch, precision, stream)


def su3_soa_to_aos_pitched(src: int, dst: int, sites: int, pitch: int, precision: int, stream: int) -> int:
    return lib.su3_soa_to_aos_pitched(src, dst, sites, pitch, precision, stream)


def su3_pack(src: int, dst: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_pack(src, dst, sites, precision, stream)


def su3_unpack(src: int, dst: int, sites: int, precision: int, stream: int) -> int:
    return lib.su3_unpack(src, dst, sites, precision, stream)


def su3_mult_nn_bwd_workspace_bytes(sites: int, precision: int) -> int:
    return lib.su3_mult_nn_bwd_workspace_bytes(sites, precision)


def su3_mult_nn_bwd(a: int, b: int, dc: int, da: int, db_f64: int, sites: int, precision: int,
                    ws: int, ws_bytes: int, stream: int) -> int:
    return lib.su3_mult_nn_bwd(a, b, dc, da, db_f64, sites, precision, ws, ws_bytes, stream)


def su3_mult_nn_bwd_noalloc(a: int, b: int, dc: int, da: int, db_f64: int, sites: int, precision: int,
                            stream: int) -> int:
    return lib.su3_mult_nn_bwd_noalloc(a, b, dc, da, db_f64, sites, precision, stream)


def su3_stream_copy(src: int, dst: int, nbytes: int, stream: int) -> int:
    return lib.su3_stream_copy(src, dst, nbytes, stream)


def su3_stream_shape(a: int, b: int, c: int, tiles: int, in_a: int, in_b: int, out: int, waves_per_cu: int,
                     tile_order: int, stream: int) -> int:
    return lib.su3_stream_shape(a, b, c, tiles, in_a, in_b, out, waves_per_cu, tile_order, stream)


def su3_launch_shape(sites: int, precision: int) -> tuple[int, int]:
    g, b = ctypes.c_int64(), ctypes.c_int()
    check(lib.su3_launch_shape(sites, precision, ctypes.byref(g), ctypes.byref(b)), "su3_launch_shape")
    return g.value, b.value
