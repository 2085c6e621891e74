"""GPU parity of the SoA layout: the AoS <-> SoA transforms are bit-exact
permutations (checked against the oracle's permutation and numpy's
transpose), and the SoA product matches the oracle's AoS product after the
same permutation (1e-13 in FP64, 5e-6 against the FP64 oracle in FP32)."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import all_finite, guards_intact, poison_, poisoned, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


@pytest.mark.parametrize("sites", [1, 63, 64, 65, 4096, 100003])
def test_transform_round_trip(O, ops, sites):
    say("aos<->soa sites=%d" % sites)
    a = latgen.random_lattice(sites, seed=sites)
    for dt in (np.complex128, np.complex64):
        x = a.astype(dt)
        s = ops.aos_to_soa(to_dev(x))
        sn = s.cpu().numpy()
        assert np.array_equal(sn, O.aos_to_soa(x))
        assert np.array_equal(sn, np.ascontiguousarray(x.transpose(1, 2, 3, 0)))
        back = ops.soa_to_aos(s).cpu().numpy()
        assert np.array_equal(back, x)


@pytest.mark.parametrize("sites", [1, 65, 4096, 100003])
def test_soa_product(O, ops, sites):
    say("fwd soa sites=%d" % sites)
    a = latgen.random_lattice(sites, seed=sites + 1)
    b = latgen.random_b(seed=3)
    ref = O.aos_to_soa(O.mult_nn(a, b))
    c = ops.mult_nn_soa(ops.aos_to_soa(to_dev(a)), to_dev(b))
    assert all_finite(c)
    assert O.max_abs_diff(c.cpu().numpy(), ref) <= 1e-13
    a32, b32 = O.round_f32(a), O.round_f32(b)
    c32 = ops.mult_nn_soa(ops.aos_to_soa(to_dev(a32)), to_dev(b32)).cpu().numpy()
    assert O.max_abs_diff(c32.astype(np.complex128), ref) <= 5e-6
    # exact pin: b = I
    ci = ops.mult_nn_soa(ops.aos_to_soa(to_dev(a)), to_dev(latgen.identity_b())).cpu().numpy()
    assert np.array_equal(ci, O.aos_to_soa(a))


def test_soa_matches_aos_at_l32(O, ops):
    say("fwd soa vs aos L=32")
    sites = 32 ** 4
    a = latgen.random_lattice(sites, seed=1)
    b = to_dev(latgen.random_b(seed=2))
    ta = to_dev(a)
    c_aos = ops.mult_nn(ta, b)
    c_soa = ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(ta), b))
    d = (torch.view_as_real(c_aos) - torch.view_as_real(c_soa)).abs().max().item()
    assert d <= 1e-13


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("shape", [(1, 0, 1), (3, 0, 3), (3, 3, 3), (6, 0, 9), (9, 0, 9)])
def test_stream_shape_pattern(ops, shape, order):
    """The access-shape probe reads and writes exactly the chunks it
    documents, in either tile order: chunk i of lane l of tile w holds the
    XOR of the lane's loaded chunks with i added to its first word. 7 tiles
    leave 7 of the 8 XCDs one tile and the last none; 19 give 3, 3, 3, 2, ..."""
    in_a, in_b, out = shape
    tiles = 7 if order == 0 else 19
    say("stream shape %s tiles=%d order=%d" % (shape, tiles, order))
    rng = np.random.default_rng(sum(shape))
    a = rng.integers(0, 2 ** 32, size=(tiles, in_a, 64, 4), dtype=np.uint32)
    b = rng.integers(0, 2 ** 32, size=(tiles, max(in_b, 1), 64, 4), dtype=np.uint32)[:, :in_b]
    x = np.bitwise_xor.reduce(np.concatenate([a, b], axis=1), axis=1)          # (tiles, 64, 4)
    want = np.repeat(x[:, None], out, axis=1)
    want[..., 0] += np.arange(out, dtype=np.uint32)[None, :, None]
    ta = to_dev(a.view(np.uint8).reshape(-1))
    tb = to_dev(np.ascontiguousarray(b).view(np.uint8).reshape(-1)) if in_b else None
    tc = torch.zeros(tiles * out * 1024, dtype=torch.uint8, device=ta.device)
    ops.stream_shape(ta, tb, tc, in_a, in_b, out, waves_per_cu=8, tile_order=order)
    got = tc.cpu().numpy().view(np.uint32).reshape(tiles, out, 64, 4)
    assert np.array_equal(got, want)


def test_stream_copy_bytes(ops):
    """The bandwidth reference copies every byte, ragged sizes included."""
    say("stream copy")
    rng = np.random.default_rng(5)
    for n in (16, 1024, 1040, 65536 * 16 + 48):
        src = to_dev(rng.integers(0, 256, size=n, dtype=np.uint8))
        dst = torch.zeros_like(src)
        ops.stream_copy(src, dst)
        assert torch.equal(src, dst)


def _abi_call(fn, *args):
    from paper_2103_00571_amd import abi
    abi.check(fn(*args, torch.cuda.current_stream().cuda_stream), fn.__name__)


@pytest.mark.parametrize("sites", [1, 65, 4096, 100003])
def test_pitched_transform_round_trip(O, ops, sites):
    """The padded SoA layout: plane p at element p * pitch. The transforms
    write the first `sites` elements of each plane bit-exactly and leave the
    padding (poisoned with NaN) untouched; the way back reads only those
    elements. Odd pitches (sites + 1) included."""
    from paper_2103_00571_amd import abi
    a = latgen.random_lattice(sites, seed=sites + 7)
    for dt, form in ((np.complex128, ops.SU3_F64), (np.complex64, ops.SU3_F32)):
        x = a.astype(dt)
        tx = to_dev(x)
        want = O.aos_to_soa(x)
        for pitch in (sites, sites + 1, ops.soa_pitch(sites, form)):
            say("aos<->soa pitched sites=%d pitch=%d form=%d" % (sites, pitch, form))
            s = poison_(torch.empty((4, 3, 3, pitch), dtype=tx.dtype, device=tx.device))
            _abi_call(abi.su3_aos_to_soa_pitched, tx.data_ptr(), s.data_ptr(), sites, pitch, form)
            sn = s.cpu().numpy()
            assert np.array_equal(sn[..., :sites], want)
            assert np.isnan(sn[..., sites:].real).all() and np.isnan(sn[..., sites:].imag).all()
            assert np.array_equal(ops.aos_to_soa(tx, pitch).cpu().numpy()[..., :sites], want)
            view, whole = poisoned((sites, 4, 3, 3), tx.dtype)
            _abi_call(abi.su3_soa_to_aos_pitched, s.data_ptr(), view.data_ptr(), sites, pitch, form)
            assert np.array_equal(view.cpu().numpy(), x)
            assert guards_intact(whole)
            assert np.array_equal(ops.soa_to_aos(s, sites).cpu().numpy(), x)


@pytest.mark.parametrize("sites", [1, 65, 4096, 100003])
def test_pitched_soa_product(O, ops, sites):
    """The product on the padded layout: bit-identical to the dense SoA
    product (same arithmetic per element), within 1e-13 of the FP64 oracle,
    5e-6 in FP32, exact for b = I, and the output's padding untouched."""
    a = latgen.random_lattice(sites, seed=sites + 11)
    b = latgen.random_b(seed=5)
    ref = O.aos_to_soa(O.mult_nn(a, b))
    for dt, form, tol in ((np.complex128, ops.SU3_F64, 1e-13), (np.complex64, ops.SU3_F32, 5e-6)):
        x = a if dt == np.complex128 else O.round_f32(a)
        bx = b if dt == np.complex128 else O.round_f32(b)
        ta, tb = to_dev(x), to_dev(bx)
        dense = ops.mult_nn_soa(ops.aos_to_soa(ta), tb).cpu().numpy()
        for pitch in (sites + 1, ops.soa_pitch(sites, form)):
            say("fwd soa pitched sites=%d pitch=%d form=%d" % (sites, pitch, form))
            sa = poison_(torch.empty((4, 3, 3, pitch), dtype=ta.dtype, device=ta.device))
            sa[..., :sites] = ops.aos_to_soa(ta)
            sc = poison_(torch.empty_like(sa))
            ops.mult_nn_soa(sa, tb, out=sc, sites=sites)
            cn = sc.cpu().numpy()
            assert np.isnan(cn[..., sites:].real).all() and np.isnan(cn[..., sites:].imag).all()
            assert np.array_equal(cn[..., :sites], dense)
            assert O.max_abs_diff(cn[..., :sites].astype(np.complex128), ref) <= tol
            ci = ops.mult_nn_soa(sa, to_dev(latgen.identity_b().astype(dt)), sites=sites).cpu().numpy()
            assert np.array_equal(ci[..., :sites], O.aos_to_soa(x))
