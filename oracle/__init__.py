"""Oracle for the SU(3) link multiply: numpy-facing wrappers around
`su3_oracle.c`, a plain single-threaded C implementation in FP64.

TEST INFRASTRUCTURE. Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module. The GPU library never
imports or links it, and it imports nothing from the GPU library.

Arrays use the site-major layout of the paper (Background / SU3_Bench):
complex128 of shape (sites, 4, 3, 3), link j of site s row-major, and
b of shape (4, 3, 3).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "su3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The multi-core CPU baseline (not the oracle): an OpenMP program that times
# the product on every host core, run as a child process by the benchmark.
_OMP_SRC = os.path.join(_HERE, "su3_cpu_omp.c")
CPU_OMP = os.path.join(_HERE, "su3_cpu_omp")
# x86-64-v3 (AVX2, FMA): any host CPU this runs on has it
OMP_CFLAGS = ["-O3", "-std=c11", "-march=x86-64-v3", "-fopenmp"]

# -ffp-contract=off: no fused multiply-add, so every rounding is the one the
# source spells out. No -ffast-math.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so, and the multi-core baseline program beside it,
    with gcc. Returns the library's path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    if force or not os.path.exists(CPU_OMP):
        tmp = CPU_OMP + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *OMP_CFLAGS, _OMP_SRC, "-o", tmp], check=True)
        os.replace(tmp, CPU_OMP)
    return _LIB


def _bind(path: str) -> ctypes.CDLL:
    lib = ctypes.CDLL(path)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "su3o_mult_nn": ([P, P, P, I64], None),
        "su3o_mult_nn_bwd": ([P, P, P, P, P, I64], None),
        "su3o_recon_row2": ([P, P, P], None),
        "su3o_max_abs_diff": ([P, P, I64], D),
        "su3o_unitarity_dev": ([P, I64], D),
        "su3o_det": ([P, P, P], None),
        "su3o_det_dev": ([P, I64], D),
        "su3o_round_f32": ([P, P, I64], None),
        "su3o_round_bf16": ([P, P, I64], None),
        "su3o_f32_to_bf16": ([P, P, I64], None),
        "su3o_widen_bf16": ([P, P, I64], None),
        "su3o_pack_r12": ([P, P, I64], None),
        "su3o_unpack_r12": ([P, P, I64], None),
        "su3o_mult_nn_f32": ([P, P, P, I64], None),
        "su3o_mult_nn_bf16": ([P, P, P, I64], None),
        "su3o_mult_nn_r12": ([P, P, P, I64], None),
        "su3o_aos_to_soa": ([P, P, I64, I32], None),
        "su3o_mult_na": ([P, P, P, I64], None),
        "su3o_mult_an": ([P, P, P, I64], None),
        "su3o_mult_nn_r12_f64": ([P, P, P, I64], None),
        "su3o_mat_vec": ([P, P, P, I64], None),
        "su3o_soa_to_aos": ([P, P, I64, I32], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load liboracle.so, compiling it first only if it is not built."""
    global _lib
    if path is not None:
        return _bind(path)
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            _lib = _bind(_LIB)
    return _lib


def _p(x: np.ndarray) -> int:
    return x.ctypes.data


def _c128(x: np.ndarray, shape_tail: tuple) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    if x.shape[-len(shape_tail):] != shape_tail:
        raise ValueError("expected trailing shape %s, got %s" % (shape_tail, x.shape))
    return x


class Oracle:
    """numpy front end of one loaded oracle library (the default one, or a
    variant compiled from another source for mutation tests)."""

    def __init__(self, lib: ctypes.CDLL | None = None):
        self.lib = lib if lib is not None else load()

    # O1 -------------------------------------------------------------------
    def mult_nn(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        a = _c128(a, (4, 3, 3))
        b = _c128(b, (4, 3, 3))
        c = np.empty_like(a)
        self.lib.su3o_mult_nn(_p(a), _p(b), _p(c), a.shape[0])
        return c

    # O2 -------------------------------------------------------------------
    def mult_nn_bwd(self, a: np.ndarray, b: np.ndarray, dc: np.ndarray):
        a = _c128(a, (4, 3, 3))
        b = _c128(b, (4, 3, 3))
        dc = _c128(dc, (4, 3, 3))
        if dc.shape != a.shape:
            raise ValueError("dc must have the shape of a")
        da = np.empty_like(a)
        db = np.empty((4, 3, 3), dtype=np.complex128)
        self.lib.su3o_mult_nn_bwd(_p(a), _p(b), _p(dc), _p(da), _p(db), a.shape[0])
        return da, db

    # O3 -------------------------------------------------------------------
    def recon_row2(self, r0: np.ndarray, r1: np.ndarray) -> np.ndarray:
        r0 = np.ascontiguousarray(r0, dtype=np.complex128).reshape(3)
        r1 = np.ascontiguousarray(r1, dtype=np.complex128).reshape(3)
        r2 = np.empty(3, dtype=np.complex128)
        self.lib.su3o_recon_row2(_p(r0), _p(r1), _p(r2))
        return r2

    # O4 -------------------------------------------------------------------
    def max_abs_diff(self, x: np.ndarray, y: np.ndarray) -> float:
        x = np.ascontiguousarray(x)
        y = np.ascontiguousarray(y)
        if x.dtype != y.dtype or x.shape != y.shape:
            raise ValueError("max_abs_diff needs equal dtype and shape")
        xr = x.astype(np.complex128).view(np.float64) if np.iscomplexobj(x) else x.astype(np.float64)
        yr = y.astype(np.complex128).view(np.float64) if np.iscomplexobj(y) else y.astype(np.float64)
        xr = np.ascontiguousarray(xr)
        yr = np.ascontiguousarray(yr)
        return float(self.lib.su3o_max_abs_diff(_p(xr), _p(yr), xr.size))

    def unitarity_dev(self, u: np.ndarray) -> float:
        u = np.ascontiguousarray(u, dtype=np.complex128)
        return float(self.lib.su3o_unitarity_dev(_p(u), u.size // 9))

    def det(self, m: np.ndarray) -> complex:
        m = np.ascontiguousarray(m, dtype=np.complex128).reshape(3, 3)
        re, im = ctypes.c_double(), ctypes.c_double()
        self.lib.su3o_det(_p(m), ctypes.byref(re), ctypes.byref(im))
        return complex(re.value, im.value)

    def det_dev(self, u: np.ndarray) -> float:
        u = np.ascontiguousarray(u, dtype=np.complex128)
        return float(self.lib.su3o_det_dev(_p(u), u.size // 9))

    # O5 -------------------------------------------------------------------
    def round_f32(self, x: np.ndarray) -> np.ndarray:
        """FP64 complex -> complex64, round to nearest even."""
        x = np.ascontiguousarray(x, dtype=np.complex128)
        out = np.empty(x.shape, dtype=np.complex64)
        self.lib.su3o_round_f32(_p(x), _p(out), 2 * x.size)
        return out

    def round_bf16(self, x: np.ndarray) -> np.ndarray:
        """FP64 complex -> BF16 bit patterns (uint16), shape x.shape + (2,)."""
        x = np.ascontiguousarray(x, dtype=np.complex128)
        out = np.empty(x.shape + (2,), dtype=np.uint16)
        self.lib.su3o_round_bf16(_p(x), _p(out), 2 * x.size)
        return out

    def f32_to_bf16(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty(x.shape, dtype=np.uint16)
        self.lib.su3o_f32_to_bf16(_p(x), _p(out), x.size)
        return out

    def widen_bf16(self, h: np.ndarray) -> np.ndarray:
        """BF16 bit patterns (..., 2) -> complex128 (...)."""
        h = np.ascontiguousarray(h, dtype=np.uint16)
        if h.shape[-1] != 2:
            raise ValueError("last axis must hold (re, im)")
        out = np.empty(h.shape[:-1], dtype=np.complex128)
        self.lib.su3o_widen_bf16(_p(h), _p(out), h.size)
        return out

    def pack_r12(self, a: np.ndarray) -> np.ndarray:
        a = _c128(a, (4, 3, 3))
        out = np.empty((a.shape[0], 4, 2, 3), dtype=np.complex64)
        self.lib.su3o_pack_r12(_p(a), _p(out), a.shape[0])
        return out

    def unpack_r12(self, a12: np.ndarray) -> np.ndarray:
        a12 = np.ascontiguousarray(a12, dtype=np.complex64)
        if a12.shape[-3:] != (4, 2, 3):
            raise ValueError("expected (sites, 4, 2, 3) complex64")
        out = np.empty((a12.shape[0], 4, 3, 3), dtype=np.complex128)
        self.lib.su3o_unpack_r12(_p(a12), _p(out), a12.shape[0])
        return out

    def mult_nn_f32(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.complex64)
        b = np.ascontiguousarray(b, dtype=np.complex64)
        c = np.empty_like(a)
        self.lib.su3o_mult_nn_f32(_p(a), _p(b), _p(c), a.shape[0])
        return c

    def mult_nn_bf16(self, a16: np.ndarray, b32: np.ndarray) -> np.ndarray:
        a16 = np.ascontiguousarray(a16, dtype=np.uint16)
        b32 = np.ascontiguousarray(b32, dtype=np.complex64)
        if a16.shape[-4:] != (4, 3, 3, 2):
            raise ValueError("expected (sites, 4, 3, 3, 2) uint16")
        c = np.empty_like(a16)
        self.lib.su3o_mult_nn_bf16(_p(a16), _p(b32), _p(c), a16.shape[0])
        return c

    def mult_nn_r12(self, a12: np.ndarray, b32: np.ndarray) -> np.ndarray:
        a12 = np.ascontiguousarray(a12, dtype=np.complex64)
        b32 = np.ascontiguousarray(b32, dtype=np.complex64)
        c = np.empty((a12.shape[0], 4, 3, 3), dtype=np.complex64)
        self.lib.su3o_mult_nn_r12(_p(a12), _p(b32), _p(c), a12.shape[0])
        return c

    # O6 -------------------------------------------------------------------
    def aos_to_soa(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x)
        sites = x.shape[0]
        out = np.empty((4, 3, 3, sites), dtype=x.dtype)
        self.lib.su3o_aos_to_soa(_p(x), _p(out), sites, x.dtype.itemsize)
        return out

    def soa_to_aos(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x)
        sites = x.shape[-1]
        out = np.empty((sites, 4, 3, 3), dtype=x.dtype)
        self.lib.su3o_soa_to_aos(_p(x), _p(out), sites, x.dtype.itemsize)
        return out

    # O7-O9 ----------------------------------------------------------------
    def mult_na(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        """c = a b^H per site and link."""
        a = _c128(a, (4, 3, 3))
        b = _c128(b, (4, 3, 3))
        c = np.empty_like(a)
        self.lib.su3o_mult_na(_p(a), _p(b), _p(c), a.shape[0])
        return c

    def mult_an(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        """c = a^H b per site and link."""
        a = _c128(a, (4, 3, 3))
        b = _c128(b, (4, 3, 3))
        c = np.empty_like(a)
        self.lib.su3o_mult_an(_p(a), _p(b), _p(c), a.shape[0])
        return c

    def mult_nn_r12_f64(self, a12: np.ndarray, b: np.ndarray) -> np.ndarray:
        """Reconstruct-12 product in FP64: a12 is (sites, 4, 2, 3)."""
        a12 = _c128(a12, (4, 2, 3))
        b = _c128(b, (4, 3, 3))
        c = np.empty((a12.shape[0], 4, 3, 3), dtype=np.complex128)
        self.lib.su3o_mult_nn_r12_f64(_p(a12), _p(b), _p(c), a12.shape[0])
        return c

    def mat_vec(self, a: np.ndarray, v: np.ndarray) -> np.ndarray:
        """w[s][j] = a[s][j] v[s]; v is (sites, 3), w is (sites, 4, 3)."""
        a = _c128(a, (4, 3, 3))
        v = np.ascontiguousarray(v, dtype=np.complex128)
        if v.shape != (a.shape[0], 3):
            raise ValueError("v must be (sites, 3)")
        w = np.empty((a.shape[0], 4, 3), dtype=np.complex128)
        self.lib.su3o_mat_vec(_p(a), _p(v), _p(w), a.shape[0])
        return w


_default: Oracle | None = None



def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
