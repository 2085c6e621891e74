"""GPU parity of the reduced storage forms against the oracle.

pack/unpack are conversions: bit-exact against the oracle's rounding.
Products: against the oracle's emulator of the same form (same inputs, same
precision; tight bound set by FMA and summation order) and against the FP64
oracle on the unrounded inputs with the forms' stated tolerances:
FP32 5e-6, reconstruct-12 1e-5, BF16 1e-2 (max abs component error)."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import L48, all_finite, bf16_bits, guards_intact, l48_case, poisoned, say, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 5e-6, "r12": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def _bf16_ulp(x):
    x = np.abs(np.asarray(x, dtype=np.float64))
    return 2.0 ** (np.floor(np.log2(np.maximum(x, 2.0 ** -126))) - 7)


# The kernel and the emulator both form each output component in FP32 from
# the same BF16 a and FP32 b, as a 6-term sum of products, but in different
# orders and with and without fused multiply-adds. Two such evaluations differ
# by at most 2 gamma_6 sum |x_i y_i| (gamma_n = n u / (1 - n u), u = 2^-24);
# for links whose rows and columns have norm at most 1 + 2^-8 the sum of
# |x_i y_i| is at most 2 (1 + 2^-8)^2, so the FP32 values differ by at most
# 1.5e-6. Each is then rounded to BF16 once, which can add at most one BF16
# ulp of the larger value. Where the sum cancels to a tiny value, that ulp is
# far below 1.5e-6, so one ulp alone is not a bound.
FP32_ORDER_BOUND = 2 * (6 * 2.0 ** -24 / (1 - 6 * 2.0 ** -24)) * 2 * (1 + 2.0 ** -8) ** 2


def _bf16_close(got, want):
    """got and want (complex128 widened from BF16) within one BF16 ulp of the
    larger magnitude plus the FP32 evaluation-order bound."""
    g, w = got.view(np.float64), want.view(np.float64)
    return np.all(np.abs(g - w) <= _bf16_ulp(np.maximum(np.abs(g), np.abs(w))) + FP32_ORDER_BOUND)


# ---------------------------------------------------------------- pack/unpack

def test_pack_unpack_bit_exact(O, ops):
    say("pack/unpack bit-exact")
    a = latgen.random_lattice(20011, seed=21)
    # add exact rounding ties: (2m+1) 2^(e-8) with 2^7 <= m < 2^8 lies halfway
    # between two BF16 values (m and m+1 ulps); (2m+1) 2^(e-24) with
    # 2^23 <= m < 2^24 lies halfway between two FP32 values. m of both
    # parities occurs, so ties to even round both up and down.
    rng = np.random.default_rng(5)
    m16 = rng.integers(1 << 7, 1 << 8, size=400)
    e16 = rng.integers(-5, 3, size=400)
    ties = (2.0 * m16 + 1.0) * np.exp2(e16 - 8.0) * rng.choice([-1.0, 1.0], size=400)
    a.reshape(-1)[:400] = ties - 1j * ties[::-1]
    m32 = rng.integers(1 << 23, 1 << 24, size=400)
    f32ties = (2.0 * m32 + 1.0) * np.exp2(rng.integers(-5, 3, size=400) - 24.0)
    a.reshape(-1)[400:800] = f32ties - 1j * f32ties[::-1]
    ta = to_dev(a)

    p32 = ops.pack(ta, ops.SU3_F32).cpu().numpy()
    assert np.array_equal(p32.view(np.uint32), O.round_f32(a).view(np.uint32))
    p16 = bf16_bits(ops.pack(ta, ops.SU3_BF16))
    assert np.array_equal(p16, O.round_bf16(a))
    p12 = ops.pack(ta, ops.SU3_R12_F32).cpu().numpy()
    assert np.array_equal(p12.view(np.uint32), O.pack_r12(a).view(np.uint32))
    p64 = ops.pack(ta, ops.SU3_F64).cpu().numpy()
    assert np.array_equal(p64, a)

    u32 = ops.unpack(ops.pack(ta, ops.SU3_F32)).cpu().numpy()
    assert np.array_equal(u32, O.round_f32(a).astype(np.complex128))
    u16 = ops.unpack(ops.pack(ta, ops.SU3_BF16)).cpu().numpy()
    assert np.array_equal(u16, O.widen_bf16(O.round_bf16(a)))
    u12 = ops.unpack(ops.pack(ta, ops.SU3_R12_F32)).cpu().numpy()
    assert np.array_equal(u12.view(np.uint64), O.unpack_r12(O.pack_r12(a)).view(np.uint64))


# ---------------------------------------------------------------- products

def _inputs(sites, seed=1):
    return latgen.random_lattice(sites, seed=seed), latgen.random_b(seed=seed + 1)


def test_f32_form(O, ops):
    say("fwd f32 L=8")
    a, b = _inputs(8 ** 4)
    a32, b32 = O.round_f32(a), O.round_f32(b)
    c = ops.mult_nn(to_dev(a32), to_dev(b32)).cpu().numpy()
    assert O.max_abs_diff(c, O.mult_nn_f32(a32, b32)) <= 1e-6
    assert O.max_abs_diff(c.astype(np.complex128), O.mult_nn(a, b)) <= TOL["f32"]
    # exact pins
    eye = latgen.identity_b().astype(np.complex64)
    assert np.array_equal(ops.mult_nn(to_dev(a32), to_dev(eye)).cpu().numpy(), a32)
    pb = latgen.permutation_b().astype(np.complex64)
    assert np.array_equal(ops.mult_nn(to_dev(a32), to_dev(pb)).cpu().numpy(), O.mult_nn_f32(a32, pb))
    pa, pbb = latgen.paper_init(999)
    c1 = ops.mult_nn(to_dev(pa.astype(np.complex64)), to_dev(pbb.astype(np.complex64))).cpu().numpy()
    assert np.all(c1 == 1.0)


def test_bf16_form(O, ops):
    say("fwd bf16 L=8")
    a, b = _inputs(8 ** 4)
    ta = to_dev(a)
    a16 = ops.pack(ta, ops.SU3_BF16)
    b32 = O.round_f32(b)
    c16 = ops.mult_nn(a16, to_dev(b32))
    bits = bf16_bits(c16)
    emu = O.mult_nn_bf16(bf16_bits(a16), b32)
    got, want = O.widen_bf16(bits), O.widen_bf16(emu)
    # FMA and FP32 summation order may move a value across a rounding
    # boundary: one BF16 ulp plus the FP32 order bound from the emulator
    assert _bf16_close(got, want)
    assert O.max_abs_diff(got, O.mult_nn(a, b)) <= TOL["bf16"]
    eye = to_dev(latgen.identity_b().astype(np.complex64))
    assert np.array_equal(bf16_bits(ops.mult_nn(a16, eye)), bf16_bits(a16))
    pa, pbb = latgen.paper_init(999)
    c1 = O.widen_bf16(bf16_bits(ops.mult_nn(ops.pack(to_dev(pa), ops.SU3_BF16),
                                            to_dev(pbb.astype(np.complex64)))))
    assert np.all(c1 == 1.0)


def test_r12_form(O, ops):
    say("fwd r12 L=8")
    a, b = _inputs(8 ** 4)
    a12 = ops.pack(to_dev(a), ops.SU3_R12_F32)
    b32 = O.round_f32(b)
    c = ops.mult_nn(a12, to_dev(b32)).cpu().numpy()
    assert O.max_abs_diff(c, O.mult_nn_r12(a12.cpu().numpy(), b32)) <= 2e-6
    assert O.max_abs_diff(c.astype(np.complex128), O.mult_nn(a, b)) <= TOL["r12"]
    eye = to_dev(latgen.identity_b().astype(np.complex64))
    ci = ops.mult_nn(a12, eye).cpu().numpy()
    assert np.array_equal(ci[:, :, :2, :], a12.cpu().numpy())


@pytest.mark.parametrize("form", ["f32", "bf16", "r12"])
@pytest.mark.parametrize("sites", [1, 2, 63, 65, 257, 4097, 65537])
def test_forms_tails_poisoned(O, ops, form, sites):
    say("fwd %s tail sites=%d" % (form, sites))
    a, b = _inputs(sites, seed=sites)
    b32 = to_dev(O.round_f32(b))
    code = {"f32": ops.SU3_F32, "bf16": ops.SU3_BF16, "r12": ops.SU3_R12_F32}[form]
    x = ops.pack(to_dev(a), code)
    shape = (sites, 4, 3, 3, 2) if form == "bf16" else (sites, 4, 3, 3)
    dtype = torch.bfloat16 if form == "bf16" else torch.complex64
    out, whole = poisoned(shape, dtype)
    ops.mult_nn(x, b32, out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole)
    assert all_finite(out)
    got = O.widen_bf16(bf16_bits(out)) if form == "bf16" else out.cpu().numpy().astype(np.complex128)
    assert O.max_abs_diff(got, O.mult_nn(a, b)) <= TOL[form]


def test_l48_forms_full(O, ops):
    """L=48 precision forms in the benchmark's launch configuration: every
    output, written into a NaN-poisoned buffer with guard sites, against the
    FP64 oracle on the unrounded inputs (FP32 5e-6, BF16 1e-2,
    reconstruct-12 1e-5) and against the oracle's emulator of the same form
    (FP32 1e-6, reconstruct-12 2e-6, BF16 one BF16 ulp plus the FP32
    evaluation-order bound)."""
    sites = L48
    say("fwd forms L=48 full")
    a, b, ref = l48_case()
    ta = to_dev(a)
    b32h = O.round_f32(b)
    b32 = to_dev(b32h)
    for name, code in (("f32", ops.SU3_F32), ("bf16", ops.SU3_BF16), ("r12", ops.SU3_R12_F32)):
        say("  form %s" % name)
        x = ops.pack(ta, code)
        shape = (sites, 4, 3, 3, 2) if name == "bf16" else (sites, 4, 3, 3)
        out, whole = poisoned(shape, torch.bfloat16 if name == "bf16" else torch.complex64)
        ops.mult_nn(x, b32, out=out)
        torch.cuda.synchronize()
        assert guards_intact(whole)
        if name == "bf16":
            bits = bf16_bits(out)
            got = O.widen_bf16(bits)
            want = O.widen_bf16(O.mult_nn_bf16(bf16_bits(x), b32h))
            assert _bf16_close(got, want)
        else:
            c = out.cpu().numpy()
            emu = O.mult_nn_f32(x.cpu().numpy(), b32h) if name == "f32" else O.mult_nn_r12(x.cpu().numpy(), b32h)
            assert O.max_abs_diff(c, emu) <= (1e-6 if name == "f32" else 2e-6)
            got = c.astype(np.complex128)
            del c, emu
        del x, out, whole
        assert O.max_abs_diff(got, ref) <= TOL[name]
        del got
