"""GPU parity of the products beyond the paper's a b: reconstruct-12 in and
out (FP32), reconstruct-12 in FP64, a b^H, a^H b, and the matrix x colour
vector product, against the oracle. Tolerances: FP64 1e-13, FP32 5e-6,
reconstruct-12 FP32 1e-5 (max abs component error vs the FP64 oracle on the
unrounded inputs)."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import L48, all_finite, guards_intact, l48_case, poison_, poisoned, say, to_dev

pytestmark = pytest.mark.gpu

TAILS = [1, 2, 3, 63, 65, 257, 4097, 65537]


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def _case(sites, seed):
    return latgen.random_lattice(sites, seed=seed), latgen.random_b(seed=seed + 1)


# ------------------------------------------------------- reconstruct-12, FP32 out compressed

@pytest.mark.parametrize("sites", TAILS)
def test_r12c_product(O, ops, sites):
    say("r12c sites=%d" % sites)
    a, b = _case(sites, sites)
    a12 = ops.pack(to_dev(a), ops.SU3_R12C_F32)
    b32 = O.round_f32(b)
    out, whole = poisoned((sites, 4, 2, 3), torch.complex64)
    ops.mult_nn(a12, to_dev(b32), out=out, form=ops.SU3_R12C_F32)
    torch.cuda.synchronize()
    assert guards_intact(whole) and all_finite(out)
    c = out.cpu().numpy()
    # rows 0-1 of the product equal those of the full reconstruct-12 emulator
    emu = O.mult_nn_r12(a12.cpu().numpy(), b32)
    assert O.max_abs_diff(c, np.ascontiguousarray(emu[:, :, :2, :])) <= 2e-6
    ref = O.mult_nn(a, b)
    assert O.max_abs_diff(c.astype(np.complex128), np.ascontiguousarray(ref[:, :, :2, :])) <= 1e-5
    # the compressed product unpacks (row 2 rebuilt) to the full product
    full = ops.unpack(out, ops.SU3_R12C_F32).cpu().numpy()
    assert O.max_abs_diff(full, ref) <= 1e-5


def test_r12c_identity_exact(O, ops):
    say("r12c identity")
    a = latgen.random_lattice(5000, seed=9)
    a12 = ops.pack(to_dev(a), ops.SU3_R12C_F32)
    c = ops.mult_nn(a12, to_dev(latgen.identity_b().astype(np.complex64)), form=ops.SU3_R12C_F32)
    assert torch.equal(torch.view_as_real(c), torch.view_as_real(a12))


# ------------------------------------------------------- reconstruct-12, FP64

@pytest.mark.parametrize("sites", TAILS)
def test_r12_f64_product(O, ops, sites):
    say("r12 f64 sites=%d" % sites)
    a, b = _case(sites, sites + 7)
    a12 = ops.pack(to_dev(a), ops.SU3_R12_F64)
    assert np.array_equal(a12.cpu().numpy(), a[:, :, :2, :])
    out, whole = poisoned((sites, 4, 3, 3), torch.complex128)
    ops.mult_nn(a12, to_dev(b), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole) and all_finite(out)
    c = out.cpu().numpy()
    assert O.max_abs_diff(c, O.mult_nn_r12_f64(a12.cpu().numpy(), b)) <= 1e-13
    assert O.max_abs_diff(c, O.mult_nn(a, b)) <= 1e-13


def test_r12_f64_unpack_bit_exact(O, ops):
    """unpack rebuilds row 2 with the oracle's operation order and no fused
    multiply-add, so it equals the oracle's rebuild bit for bit."""
    say("r12 f64 unpack")
    a = latgen.random_lattice(20000, seed=13)
    a12 = ops.pack(to_dev(a), ops.SU3_R12_F64)
    u = ops.unpack(a12).cpu().numpy()
    ref = O.mult_nn_r12_f64(a12.cpu().numpy(), latgen.identity_b())
    assert np.array_equal(u.view(np.uint64), ref.view(np.uint64))


# ------------------------------------------------------- a b^H and a^H b

@pytest.mark.parametrize("sites", TAILS)
@pytest.mark.parametrize("op", ["na", "an"])
def test_na_an(O, ops, op, sites):
    say("%s sites=%d" % (op, sites))
    a, b = _case(sites, sites + 21)
    fn = ops.mult_na if op == "na" else ops.mult_an
    ref = (O.mult_na if op == "na" else O.mult_an)(a, b)
    out, whole = poisoned((sites, 4, 3, 3), torch.complex128)
    fn(to_dev(a), to_dev(b), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole) and all_finite(out)
    assert O.max_abs_diff(out.cpu().numpy(), ref) <= 1e-13
    out32, whole32 = poisoned((sites, 4, 3, 3), torch.complex64)
    fn(to_dev(O.round_f32(a)), to_dev(O.round_f32(b)), out=out32)
    torch.cuda.synchronize()
    assert guards_intact(whole32) and all_finite(out32)
    assert O.max_abs_diff(out32.cpu().numpy().astype(np.complex128), ref) <= 5e-6


def test_na_an_exact_pins(O, ops):
    say("na/an exact pins")
    a = latgen.random_lattice(3000, seed=31)
    ta = to_dev(a)
    eye = to_dev(latgen.identity_b())
    assert np.array_equal(ops.mult_na(ta, eye).cpu().numpy(), a)
    assert np.array_equal(ops.mult_an(ta, eye).cpu().numpy(), np.conj(np.swapaxes(a, 2, 3)))
    pb = latgen.permutation_b()
    assert np.array_equal(ops.mult_na(ta, to_dev(pb)).cpu().numpy(), O.mult_na(a, pb))
    assert np.array_equal(ops.mult_an(ta, to_dev(pb)).cpu().numpy(), O.mult_an(a, pb))


def test_na_an_l32(O, ops):
    say("na/an L=32")
    sites = 32 ** 4
    a, b = _case(sites, 1)
    ta, tb = to_dev(a), to_dev(b)
    assert O.max_abs_diff(ops.mult_na(ta, tb).cpu().numpy(), O.mult_na(a, b)) <= 1e-13
    assert O.max_abs_diff(ops.mult_an(ta, tb).cpu().numpy(), O.mult_an(a, b)) <= 1e-13


# ------------------------------------------------------- matrix x colour vector

def _vec(sites, seed):
    return latgen.complex_normal_lattice(sites, seed=seed)[:, 0, 0, :].copy()


@pytest.mark.parametrize("sites", TAILS)
def test_mat_vec(O, ops, sites):
    say("mat_vec sites=%d" % sites)
    a, _ = _case(sites, sites + 41)
    v = _vec(sites, sites + 43)
    ref = O.mat_vec(a, v)
    out, whole = poisoned((sites, 4, 3), torch.complex128)
    ops.mat_vec(to_dev(a), to_dev(v), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole) and all_finite(out)
    assert O.max_abs_diff(out.cpu().numpy(), ref) <= 1e-13
    # FP32: an odd site count leaves the last colour vector straddling a
    # 16-byte boundary, which the kernel reads as 8-byte words
    out32, whole32 = poisoned((sites, 4, 3), torch.complex64)
    ops.mat_vec(to_dev(O.round_f32(a)), to_dev(O.round_f32(v)), out=out32)
    torch.cuda.synchronize()
    assert guards_intact(whole32) and all_finite(out32)
    assert O.max_abs_diff(out32.cpu().numpy().astype(np.complex128), ref) <= 5e-6


def test_mat_vec_exact_pins(O, ops):
    say("mat_vec exact pins")
    sites = 999
    v = _vec(sites, 5)
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), (sites, 4, 3, 3)).copy()
    w = ops.mat_vec(to_dev(eye), to_dev(v)).cpu().numpy()
    assert np.array_equal(w, np.broadcast_to(v[:, None, :], (sites, 4, 3)))
    a = latgen.index_coded(sites)
    e0 = np.zeros((sites, 3), dtype=np.complex128)
    e0[:, 1] = 1.0
    w = ops.mat_vec(to_dev(a), to_dev(e0)).cpu().numpy()   # picks column 1 of every link
    assert np.array_equal(w, a[:, :, :, 1])


def test_mat_vec_l48_full(O, ops):
    """L=48 matrix x colour vector: every output, written into a NaN-poisoned
    buffer with guard sites, against the oracle at 1e-13."""
    sites = L48
    say("mat_vec L=48 full")
    a, _, _ = l48_case()
    v = _vec(sites, 3)
    out, whole = poisoned((sites, 4, 3), torch.complex128)
    ops.mat_vec(to_dev(a), to_dev(v), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole)
    assert O.max_abs_diff(out.cpu().numpy(), O.mat_vec(a, v)) <= 1e-13


def test_l48_products_full(O, ops):
    """L=48 (5,308,416 sites), the inputs and launch configuration the
    benchmark times: a b^H, a^H b, reconstruct-12 in and out, reconstruct-12
    in FP64, the SoA product (FP64 and FP32, dense and at the padded pitch),
    and the FP64 product on one GPU's share of the lattice split over 8 GPUs
    (the first 663,552 sites). Every output is written into a NaN-poisoned
    buffer (with guard sites where the layout is site-major) and compared
    with the oracle."""
    sites = L48
    a, b, ref = l48_case()
    ta, tb = to_dev(a), to_dev(b)

    def run(fn, shape, dtype):
        out, whole = poisoned(shape, dtype)
        fn(out)
        torch.cuda.synchronize()
        assert guards_intact(whole)
        return out.cpu().numpy()

    full = (sites, 4, 3, 3)
    say("L=48 a b^H")
    got = run(lambda o: ops.mult_na(ta, tb, out=o), full, torch.complex128)
    assert O.max_abs_diff(got, O.mult_na(a, b)) <= 1e-13
    say("L=48 a^H b")
    got = run(lambda o: ops.mult_an(ta, tb, out=o), full, torch.complex128)
    assert O.max_abs_diff(got, O.mult_an(a, b)) <= 1e-13
    say("L=48 reconstruct-12 FP64")
    x = ops.pack(ta, ops.SU3_R12_F64)
    got = run(lambda o: ops.mult_nn(x, tb, out=o), full, torch.complex128)
    del x
    assert O.max_abs_diff(got, ref) <= 1e-13
    say("L=48 reconstruct-12 in and out")
    b32 = to_dev(O.round_f32(b))
    x = ops.pack(ta, ops.SU3_R12C_F32)
    got = run(lambda o: ops.mult_nn(x, b32, out=o, form=ops.SU3_R12C_F32), (sites, 4, 2, 3), torch.complex64)
    del x
    assert O.max_abs_diff(got.astype(np.complex128), np.ascontiguousarray(ref[:, :, :2, :])) <= 1e-5
    say("L=48 SoA")
    sa = ops.aos_to_soa(ta)
    sc = poison_(torch.empty_like(sa))
    ops.mult_nn_soa(sa, tb, out=sc)
    del sa
    got = ops.soa_to_aos(sc).cpu().numpy()
    del sc
    assert O.max_abs_diff(got, ref) <= 1e-13
    say("L=48 SoA, padded pitch")
    pitch = ops.soa_pitch(sites, ops.SU3_F64)
    sa = ops.aos_to_soa(ta, pitch)
    sc = poison_(torch.empty_like(sa))
    ops.mult_nn_soa(sa, tb, out=sc, sites=sites)
    del sa
    pad = torch.view_as_real(sc[..., sites:])
    assert bool(torch.isnan(pad).all())
    del pad
    got = ops.soa_to_aos(sc, sites).cpu().numpy()
    del sc
    assert O.max_abs_diff(got, ref) <= 1e-13
    # FP32 SoA (the dense layout loads its planes in two phases at this
    # stride; the padded one in one), every output against the FP64 oracle on
    # the unrounded inputs at the FP32 tolerance
    t32, b32 = ta.to(torch.complex64), tb.to(torch.complex64)
    for pitch in (sites, ops.soa_pitch(sites, ops.SU3_F32)):
        say("L=48 SoA FP32, pitch %d" % pitch)
        sa = ops.aos_to_soa(t32, pitch)
        sc = poison_(torch.empty_like(sa))
        ops.mult_nn_soa(sa, b32, out=sc, sites=sites)
        del sa
        if pitch > sites:
            assert bool(torch.isnan(torch.view_as_real(sc[..., sites:])).all())
        got = ops.soa_to_aos(sc, sites).cpu().numpy()
        del sc
        assert O.max_abs_diff(got.astype(np.complex128), ref) <= 5e-6
    del t32
    say("L=48 / 8 share")
    ns = sites // 8
    got = run(lambda o: ops.mult_nn(ta[:ns], tb, out=o), (ns, 4, 3, 3), torch.complex128)
    assert O.max_abs_diff(got, ref[:ns]) <= 1e-13
