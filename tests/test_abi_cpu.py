"""The C ABI on the CPU: libsu3.so loads, exports every function that
include/su3.h declares, and rejects bad arguments before any HIP call (no
pointer below is ever dereferenced; no GPU is needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "su3.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(su3_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_2103_00571_amd import abi
    return abi


def test_header_matches_library_exports(abi):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(abi.lib, n), "libsu3.so lacks %s" % n
        assert n in abi.SIGNATURES, "binding lacks %s" % n
        assert callable(getattr(abi, n)), "binding lacks a same-named wrapper for %s" % n
    assert sorted(abi.SIGNATURES) == names


def test_header_constants_match_binding(abi):
    text = open(HEADER).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"\b(SU3_[A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    for k, v in consts.items():
        assert getattr(abi, k) == v, k
    assert int(re.search(r"#define SU3_ABI_VERSION (\d+)", text).group(1)) == abi.su3_abi_version()


def test_status_strings(abi):
    for code in range(0, -8, -1):
        s = abi.su3_status_string(code)
        assert s.startswith("SU3_")
    assert "unknown" in abi.su3_status_string(42)


# 16-byte aligned fake device addresses, far apart. Every call below must be
# rejected (or be a no-op for zero sites) before any HIP call: none of them
# may pass validation, or it would launch a kernel on these addresses.
A, B, C = 1 << 20, 1 << 30, 1 << 40


@pytest.mark.parametrize("form", [0, 1, 2, 3, 4, 5])
def test_mult_nn_validation(abi, form):
    f = abi.su3_mult_nn
    assert f(A, B, C, 0, form, None) == abi.SU3_OK            # nothing to do: no launch
    assert f(A, B, C, -1, form, None) == abi.SU3_ERR_SIZE
    assert f(A, B, C, 1 << 62, form, None) == abi.SU3_ERR_SIZE
    assert f(0, B, C, 5, form, None) == abi.SU3_ERR_NULL
    assert f(A, 0, C, 5, form, None) == abi.SU3_ERR_NULL
    assert f(A, B, 0, 5, form, None) == abi.SU3_ERR_NULL
    assert f(A + 8, B, C, 5, form, None) == abi.SU3_ERR_ALIGN
    assert f(A, B, C + 4, 5, form, None) == abi.SU3_ERR_ALIGN
    assert f(A, B + 2, C, 5, form, None) == abi.SU3_ERR_ALIGN
    assert f(A, B, A, 5, form, None) == abi.SU3_ERR_OVERLAP            # in place
    assert f(A, B, A + 16 * 7, 5, form, None) == abi.SU3_ERR_OVERLAP   # partial overlap
    assert f(A, C + 32, C, 5, form, None) == abi.SU3_ERR_OVERLAP       # c covers b
    assert f(A, B, C, 5, 6, None) == abi.SU3_ERR_PRECISION
    assert f(A, B, C, 5, -1, None) == abi.SU3_ERR_PRECISION


@pytest.mark.parametrize("name", ["su3_mult_na", "su3_mult_an"])
def test_na_an_validation(abi, name):
    f = getattr(abi, name)
    for form in (2, 3, 4, 5, 6):
        assert f(A, B, C, 5, form, None) == abi.SU3_ERR_PRECISION
    for form in (0, 1):
        assert f(A, B, C, 0, form, None) == abi.SU3_OK
        assert f(A, B, C, -2, form, None) == abi.SU3_ERR_SIZE
        assert f(0, B, C, 5, form, None) == abi.SU3_ERR_NULL
        assert f(A + 4, B, C, 5, form, None) == abi.SU3_ERR_ALIGN
        assert f(A, B, A + 32, 5, form, None) == abi.SU3_ERR_OVERLAP


def test_mat_vec_validation(abi):
    f = abi.su3_mat_vec
    V = 1 << 35
    assert f(A, V, C, 0, 0, None) == abi.SU3_OK
    assert f(A, V, C, 5, 2, None) == abi.SU3_ERR_PRECISION
    assert f(A, V, C, -1, 0, None) == abi.SU3_ERR_SIZE
    assert f(A, 0, C, 5, 0, None) == abi.SU3_ERR_NULL
    assert f(A, V + 4, C, 5, 1, None) == abi.SU3_ERR_ALIGN      # v needs 8 bytes
    assert f(A, V, C + 8, 5, 0, None) == abi.SU3_ERR_ALIGN      # w needs 16
    assert f(A, V, A + 64, 5, 0, None) == abi.SU3_ERR_OVERLAP   # w over a
    assert f(A, V, V + 16, 5, 1, None) == abi.SU3_ERR_OVERLAP   # w over v


def test_soa_transform_pack_validation(abi):
    for f in (abi.su3_mult_nn_soa,):
        assert f(A, B, C, 5, 2, None) == abi.SU3_ERR_PRECISION
        assert f(A, B, C, 5, 3, None) == abi.SU3_ERR_PRECISION
        assert f(A, B, A, 5, 0, None) == abi.SU3_ERR_OVERLAP
    for f in (abi.su3_aos_to_soa, abi.su3_soa_to_aos):
        assert f(A, C, 0, 0, None) == abi.SU3_OK
        assert f(A, C, 5, 2, None) == abi.SU3_ERR_PRECISION
        assert f(A, A + 16, 5, 0, None) == abi.SU3_ERR_OVERLAP
        assert f(A, C + 8, 5, 1, None) == abi.SU3_ERR_ALIGN
        assert f(0, C, 5, 0, None) == abi.SU3_ERR_NULL
    for f in (abi.su3_aos_to_soa_pitched, abi.su3_soa_to_aos_pitched):
        assert f(A, C, 0, 0, 0, None) == abi.SU3_OK
        assert f(A, C, 0, 64, 0, None) == abi.SU3_OK                 # no sites: no launch
        assert f(A, C, 5, 4, 0, None) == abi.SU3_ERR_SIZE            # pitch < sites
        assert f(A, C, -1, 4, 0, None) == abi.SU3_ERR_SIZE
        assert f(A, C, 5, 1 << 62, 0, None) == abi.SU3_ERR_SIZE
        assert f(A, C, 5, 8, 2, None) == abi.SU3_ERR_PRECISION
        assert f(A, C + 8, 5, 8, 1, None) == abi.SU3_ERR_ALIGN
        assert f(0, C, 5, 8, 0, None) == abi.SU3_ERR_NULL
    # The SoA side spans 36 * pitch elements: a destination just past the 5
    # AoS sites still lies inside the padded SoA source.
    assert abi.su3_soa_to_aos_pitched(A, A + 36 * 5 * 16, 5, 64, 0, None) == abi.SU3_ERR_OVERLAP
    assert abi.su3_aos_to_soa_pitched(A + 36 * 5 * 16, A, 5, 64, 0, None) == abi.SU3_ERR_OVERLAP
    f = abi.su3_mult_nn_soa_pitched
    assert f(A, B, C, 0, 0, 0, None) == abi.SU3_OK
    assert f(A, B, C, 5, 4, 0, None) == abi.SU3_ERR_SIZE
    assert f(A, B, C, 5, 1 << 62, 1, None) == abi.SU3_ERR_SIZE
    assert f(A, B, C, 5, 8, 2, None) == abi.SU3_ERR_PRECISION
    assert f(0, B, C, 5, 8, 0, None) == abi.SU3_ERR_NULL
    assert f(A, B, C + 8, 5, 8, 0, None) == abi.SU3_ERR_ALIGN
    assert f(A, B, A + 36 * 5 * 16, 5, 64, 0, None) == abi.SU3_ERR_OVERLAP   # c inside a's padding
    assert f(A, C + 16, C, 5, 64, 1, None) == abi.SU3_ERR_OVERLAP             # c covers b
    for f in (abi.su3_pack, abi.su3_unpack):
        assert f(A, C, -3, 1, None) == abi.SU3_ERR_SIZE
        assert f(A, C, 5, 6, None) == abi.SU3_ERR_PRECISION
        assert f(A, C, 5, 7, None) == abi.SU3_ERR_PRECISION
        assert f(A, A + 64, 5, 1, None) == abi.SU3_ERR_OVERLAP
        assert f(A, 0, 5, 1, None) == abi.SU3_ERR_NULL


def test_soa_pitch(abi):
    # sites rounded up to 64, plus 512 (FP64) or 128 (FP32) elements
    for sites, p64, p32 in ((0, 512, 128), (1, 576, 192), (64, 576, 192), (65, 640, 256),
                            (1 << 20, (1 << 20) + 512, (1 << 20) + 128), (48 ** 4, 48 ** 4 + 512, 48 ** 4 + 128)):
        assert abi.su3_soa_pitch(sites, 0) == p64
        assert abi.su3_soa_pitch(sites, 1) == p32
    for sites in range(0, 3000, 37):
        p = abi.su3_soa_pitch(sites, 0)
        assert p >= sites and p % 64 == 0
    with pytest.raises(abi.SU3Error):
        abi.su3_soa_pitch(10, 2)
    with pytest.raises(abi.SU3Error):
        abi.su3_soa_pitch(-1, 0)
    assert abi.lib.su3_soa_pitch(10, 0, None) == abi.SU3_ERR_NULL


def test_bwd_validation(abi):
    ws_need = abi.su3_mult_nn_bwd_workspace_bytes(1000, 0)
    assert ws_need > 0 and ws_need % 16 == 0
    assert abi.su3_mult_nn_bwd_workspace_bytes(1000, 2) == 0
    assert abi.su3_mult_nn_bwd_workspace_bytes(0, 0) == 0
    # the workspace (72 FP64 partials per stage-1 workgroup) is a function of
    # the size and form only -- queried here with no GPU present -- and grows
    # with the lattice
    for form in (0, 1):
        w = [abi.su3_mult_nn_bwd_workspace_bytes(n, form) for n in (1, 10 ** 4, 10 ** 7)]
        assert all(x % (72 * 8) == 0 for x in w) and w[0] <= w[1] <= w[2]
        assert w == [abi.su3_mult_nn_bwd_workspace_bytes(n, form) for n in (1, 10 ** 4, 10 ** 7)]
    D, DA, DB, WS = 1 << 41, 1 << 42, 1 << 43, 1 << 44
    f = abi.su3_mult_nn_bwd
    assert f(A, B, D, DA, DB, 1000, 2, WS, ws_need, None) == abi.SU3_ERR_PRECISION
    assert f(A, B, D, DA, DB, 1000, 0, WS, ws_need - 8, None) == abi.SU3_ERR_WORKSPACE
    assert f(A, B, D, DA, DB, 1000, 0, 0, ws_need, None) == abi.SU3_ERR_WORKSPACE
    assert f(A, B, D, DA, 0, 1000, 0, WS, ws_need, None) == abi.SU3_ERR_NULL
    assert f(A, B, D, A, DB, 1000, 0, WS, ws_need, None) == abi.SU3_ERR_OVERLAP
    assert f(A, B, D, DA, DA + 64, 1000, 0, WS, ws_need, None) == abi.SU3_ERR_OVERLAP
    assert f(A, B, D, DA, DB, 1000, 0, D, ws_need, None) == abi.SU3_ERR_OVERLAP
    assert f(A, B, D, DA + 8, DB, 1000, 0, WS, ws_need, None) == abi.SU3_ERR_ALIGN
    assert f(A, B, D, DA, DB, -1, 0, WS, ws_need, None) == abi.SU3_ERR_SIZE


def test_bwd_noalloc_validation(abi):
    """The allocation-free adjoint validates like su3_mult_nn_bwd, and refuses
    a lattice whose workspace exceeds the library's array, before any HIP call
    (so before the array's address is even looked up)."""
    D, DA, DB = 1 << 41, 1 << 42, 1 << 43
    f = abi.su3_mult_nn_bwd_noalloc
    assert abi.SU3_BWD_SCRATCH_BYTES == 64 << 20
    for form in (0, 1):
        big = 1
        while abi.su3_mult_nn_bwd_workspace_bytes(big, form) <= abi.SU3_BWD_SCRATCH_BYTES:
            big *= 2
        assert f(A, B, D, DA, DB, big, form, None) == abi.SU3_ERR_WORKSPACE
        assert abi.su3_mult_nn_bwd_workspace_bytes(48 ** 4, form) <= abi.SU3_BWD_SCRATCH_BYTES
        assert f(A, B, D, DA, DB, -1, form, None) == abi.SU3_ERR_SIZE
        assert f(A, B, D, DA, 0, 1000, form, None) == abi.SU3_ERR_NULL
        assert f(0, B, D, DA, DB, 1000, form, None) == abi.SU3_ERR_NULL
        assert f(A, B, D, A, DB, 1000, form, None) == abi.SU3_ERR_OVERLAP
        assert f(A, B, D, DA, DA + 64, 1000, form, None) == abi.SU3_ERR_OVERLAP
        assert f(A, B, D, DA + 8, DB, 1000, form, None) == abi.SU3_ERR_ALIGN
    assert f(A, B, D, DA, DB, 1000, 2, None) == abi.SU3_ERR_PRECISION


def test_stream_copy_validation(abi):
    assert abi.su3_stream_copy(A, C, 0, None) == abi.SU3_OK
    assert abi.su3_stream_copy(A, C, 24, None) == abi.SU3_ERR_SIZE
    assert abi.su3_stream_copy(A, A + 16, 64, None) == abi.SU3_ERR_OVERLAP
    assert abi.su3_stream_copy(A + 4, C, 64, None) == abi.SU3_ERR_ALIGN


def test_stream_shape_validation(abi):
    f = abi.su3_stream_shape
    assert f(A, 0, C, 0, 3, 0, 3, 0, 0, None) == abi.SU3_OK                 # nothing to do
    assert f(A, 0, C, 4, 2, 0, 2, 0, 0, None) == abi.SU3_ERR_SIZE           # not a kernel's shape
    assert f(A, 0, C, -1, 3, 0, 3, 0, 0, None) == abi.SU3_ERR_SIZE
    assert f(A, 0, C, 4, 3, 0, 3, 33, 0, None) == abi.SU3_ERR_SIZE
    assert f(A, 0, C, 4, 3, 0, 3, 0, 2, None) == abi.SU3_ERR_SIZE       # tile order 0 or 1
    assert f(A, 0, C, 4, 3, 0, 3, 0, -1, None) == abi.SU3_ERR_SIZE
    assert f(A, 0, C, 1 << 26, 3, 0, 3, 0, 0, None) == abi.SU3_ERR_SIZE      # grid beyond 2^32 work-items
    assert f(A, 0, C, (1 << 62) // 1024, 9, 0, 9, 0, 0, None) == abi.SU3_ERR_SIZE   # sizes would overflow
    assert f(A, 0, C, (1 << 63) - 1, 9, 0, 9, 0, 0, None) == abi.SU3_ERR_SIZE      # so would the grid product
    assert f(0, 0, C, 4, 3, 0, 3, 0, 0, None) == abi.SU3_ERR_NULL
    assert f(A, 0, C, 4, 3, 3, 3, 0, 0, None) == abi.SU3_ERR_NULL           # b needed
    assert f(A + 8, 0, C, 4, 3, 0, 3, 0, 0, None) == abi.SU3_ERR_ALIGN
    assert f(A, B + 8, C, 4, 3, 3, 3, 0, 0, None) == abi.SU3_ERR_ALIGN
    assert f(A, 0, A + 1024, 4, 3, 0, 3, 0, 0, None) == abi.SU3_ERR_OVERLAP
    assert f(A, C + 16, C, 4, 3, 3, 3, 0, 0, None) == abi.SU3_ERR_OVERLAP


def test_launch_shape_rejects_before_hip(abi):
    g, b = ctypes.c_int64(), ctypes.c_int()
    assert abi.lib.su3_launch_shape(10, 9, ctypes.byref(g), ctypes.byref(b)) == abi.SU3_ERR_PRECISION
    assert abi.lib.su3_launch_shape(-1, 0, ctypes.byref(g), ctypes.byref(b)) == abi.SU3_ERR_SIZE
    assert abi.lib.su3_launch_shape(10, 0, None, None) == abi.SU3_ERR_NULL


def test_torch_front_end_rejects_cpu_and_bad_shapes():
    import torch
    from paper_2103_00571_amd import ops
    a = torch.zeros((3, 4, 3, 3), dtype=torch.complex128)
    b = torch.zeros((4, 3, 3), dtype=torch.complex128)
    with pytest.raises(ValueError):
        ops.mult_nn(a, b)                       # CPU tensors: never computed on the host
    with pytest.raises(ValueError):
        ops.mult_nn(a, b.to(torch.complex64))   # b dtype must match the form
    with pytest.raises(ValueError):
        ops.form_of(torch.zeros((3, 4, 3, 2), dtype=torch.complex128))
    assert ops.form_of(torch.zeros((3, 4, 2, 3), dtype=torch.complex64)) == ops.SU3_R12_F32
    assert ops.form_of(torch.zeros((3, 4, 3, 3, 2), dtype=torch.bfloat16)) == ops.SU3_BF16


def test_torch_front_end_soa_arguments():
    """The padded-SoA arguments of the torch front end are checked before any
    allocation on, or call to, the GPU."""
    import torch
    from paper_2103_00571_amd import ops
    x = torch.zeros((10, 4, 3, 3), dtype=torch.complex128)
    s = torch.zeros((4, 3, 3, 16), dtype=torch.complex128)
    b = torch.zeros((4, 3, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="pitch"):
        ops.aos_to_soa(x, pitch=9)               # pitch below the site count
    with pytest.raises(ValueError, match="sites"):
        ops.soa_to_aos(s, sites=17)              # more sites than the pitch holds
    with pytest.raises(ValueError, match="sites"):
        ops.soa_to_aos(s, sites=-1)
    with pytest.raises(ValueError, match="sites"):
        ops.mult_nn_soa(s, b, sites=17)
    with pytest.raises(ValueError):
        ops.mult_nn_soa(s, b, sites=10)          # CPU tensors: never computed on the host
    with pytest.raises(ValueError):
        ops.mult_nn_soa(s, b.to(torch.complex64), sites=10)
    with pytest.raises(ValueError):
        ops.mult_nn_soa(s, b, out=torch.zeros((4, 3, 3, 15), dtype=torch.complex128), sites=10)
    assert ops.soa_pitch(10, ops.SU3_F64) == 576 and ops.soa_pitch(10, ops.SU3_F32) == 192
