"""GPU parity of the FP64 site-major forward kernel (su3_mult_nn, SU3_F64)
against the oracle. Tolerance: 1e-13 absolute per real component."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import L48, all_finite, dev, guards_intact, l48_case, poisoned, say, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-13


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def test_l8_random_su3(O, ops):
    say("fwd f64 L=8 random SU(3)")
    a = latgen.random_lattice(8 ** 4, seed=1)
    b = latgen.random_b(seed=2)
    c = ops.mult_nn(to_dev(a), to_dev(b)).cpu().numpy()
    ref = O.mult_nn(a, b)
    assert O.max_abs_diff(c, ref) <= TOL64
    assert O.unitarity_dev(c) <= 1e-13 and O.det_dev(c) <= 1e-13


def test_exact_pins(O, ops):
    """b = I gives c == a; b = (I, P, P^2, diag(i, i, -1)) permutes columns
    exactly; the paper's init gives c = 1 exactly."""
    say("fwd f64 exact pins")
    a = latgen.random_lattice(5000, seed=3)
    ta = to_dev(a)
    c = ops.mult_nn(ta, to_dev(latgen.identity_b())).cpu().numpy()
    assert np.array_equal(c, a)
    c = ops.mult_nn(ta, to_dev(latgen.permutation_b())).cpu().numpy()
    assert np.array_equal(c, O.mult_nn(a, latgen.permutation_b()))
    pa, pb = latgen.paper_init(5000)
    c = ops.mult_nn(to_dev(pa), to_dev(pb)).cpu().numpy()
    assert np.all(c == 1.0 + 0.0j)


def test_index_coded_input_is_exact(O, ops):
    """Integer-valued entries with a permutation b: every output is an exact
    copy of one input entry, so any site, link or row slip shows up."""
    say("fwd f64 index coded")
    a = latgen.index_coded(3001)
    b = latgen.permutation_b()
    c = ops.mult_nn(to_dev(a), to_dev(b)).cpu().numpy()
    assert np.array_equal(c, O.mult_nn(a, b))


@pytest.mark.parametrize("sites", [1, 2, 3, 63, 64, 65, 255, 257, 4097, 65537])
def test_tails_poisoned_and_guarded(O, ops, sites):
    say("fwd f64 tail sites=%d" % sites)
    a = latgen.random_lattice(sites, seed=sites)
    b = latgen.random_b(seed=7)
    out, whole = poisoned((sites, 4, 3, 3), torch.complex128)
    ops.mult_nn(to_dev(a), to_dev(b), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole)
    assert all_finite(out)
    assert O.max_abs_diff(out.cpu().numpy(), O.mult_nn(a, b)) <= TOL64


def test_zero_sites(ops):
    say("fwd f64 zero sites")
    a = torch.empty((0, 4, 3, 3), dtype=torch.complex128, device=dev())
    b = to_dev(latgen.random_b())
    c = ops.mult_nn(a, b)
    assert c.shape == (0, 4, 3, 3)


def test_site_locality(O, ops):
    say("fwd f64 site locality")
    a = latgen.random_lattice(1000, seed=9)
    b = to_dev(latgen.random_b(seed=10))
    c0 = ops.mult_nn(to_dev(a), b).cpu().numpy()
    a[517, 3, 2, 1] += 0.25
    c1 = ops.mult_nn(to_dev(a), b).cpu().numpy()
    changed = np.argwhere(c0 != c1)
    assert set(changed[:, 0]) == {517} and set(changed[:, 1]) == {3} and set(changed[:, 2]) == {2}


def test_deterministic_and_non_default_stream(O, ops):
    say("fwd f64 determinism / side stream")
    a = to_dev(latgen.random_lattice(100003, seed=11))
    b = to_dev(latgen.random_b(seed=12))
    c0 = ops.mult_nn(a, b)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        c1 = ops.mult_nn(a, b)
    torch.cuda.current_stream().wait_stream(s)
    c2 = ops.mult_nn(a, b)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(c0), torch.view_as_real(c1))
    assert torch.equal(torch.view_as_real(c0), torch.view_as_real(c2))


def test_l32_full_parity(O, ops):
    """configs: L=32, 1,048,576 sites, every output compared."""
    say("fwd f64 L=32 full parity")
    sites = 32 ** 4
    a = latgen.random_lattice(sites, seed=1)
    b = latgen.random_b(seed=2)
    c = ops.mult_nn(to_dev(a), to_dev(b)).cpu().numpy()
    assert O.max_abs_diff(c, O.mult_nn(a, b)) <= TOL64


def test_l48_full_parity_and_closure(O, ops):
    """L=48, 5,308,416 sites, in the launch configuration the benchmark times:
    every output, written into a NaN-poisoned buffer with guard sites, against
    the oracle at 1e-13, and SU(3) closure of every output (unitarity and det
    to 1e-13)."""
    sites = L48
    grid, block = ops.launch_shape(sites, ops.SU3_F64)
    say("fwd f64 L=48 full parity grid=%d block=%d" % (grid, block))
    a, b, ref = l48_case()
    out, whole = poisoned((sites, 4, 3, 3), torch.complex128)
    ops.mult_nn(to_dev(a), to_dev(b), out=out)
    torch.cuda.synchronize()
    assert guards_intact(whole)
    c = out.cpu().numpy()
    del out, whole
    assert O.max_abs_diff(c, ref) <= TOL64
    assert O.unitarity_dev(c) <= 1e-13
    assert O.det_dev(c) <= 1e-13


def test_zero_b_gives_zero(ops):
    """Degenerate b = 0: every product is exactly zero, in every form."""
    say("fwd zero b")
    a = latgen.random_lattice(4099, seed=71)
    ta = to_dev(a)
    z64 = torch.zeros((4, 3, 3), dtype=torch.complex128, device=dev())
    z32 = z64.to(torch.complex64)
    assert torch.count_nonzero(torch.view_as_real(ops.mult_nn(ta, z64))).item() == 0
    for code in (ops.SU3_F32, ops.SU3_BF16, ops.SU3_R12_F32, ops.SU3_R12C_F32):
        c = ops.mult_nn(ops.pack(ta, code), z32, form=code)
        r = c.float() if c.dtype == torch.bfloat16 else torch.view_as_real(c)
        assert torch.count_nonzero(r).item() == 0
    c = ops.mult_nn(ops.pack(ta, ops.SU3_R12_F64), z64)
    assert torch.count_nonzero(torch.view_as_real(c)).item() == 0


def test_non_finite_input_stays_in_its_row(O, ops):
    """A NaN and an infinity in a[s] reach only the output rows that read
    them; every other output is finite and matches the oracle."""
    say("fwd non-finite locality")
    a = latgen.random_lattice(2000, seed=72)
    b = latgen.random_b(seed=73)
    a[123, 1, 2, 0] = complex(float("nan"), 0.0)
    a[1500, 3, 0, 2] = complex(0.0, float("inf"))
    c = ops.mult_nn(to_dev(a), to_dev(b)).cpu().numpy()
    bad = ~np.isfinite(c.view(np.float64).reshape(2000, 4, 3, 3, 2)).all(axis=(3, 4))
    assert set(map(tuple, np.argwhere(bad))) == {(123, 1, 2), (1500, 3, 0)}
    keep = np.ones(2000, dtype=bool)
    keep[[123, 1500]] = False
    ref = O.mult_nn(a[keep], b)
    assert O.max_abs_diff(c[keep], ref) <= TOL64


def test_hand_expanded_2_4_lattice(ops):
    """The GPU product on a 2^4 lattice against the 3x3 products written out
    entry by entry (c_kl = a_k0 b_0l + a_k1 b_1l + a_k2 b_2l)."""
    say("fwd f64 hand-expanded 2^4")
    from test_oracle_pins import _hand_expanded
    a = latgen.random_lattice(2 ** 4, seed=131)
    b = latgen.random_b(seed=132)
    c = ops.mult_nn(to_dev(a), to_dev(b)).cpu().numpy()
    assert np.abs(c - _hand_expanded(a, b)).max() <= 1e-15


def test_lazy_conjugate_views_are_rejected(ops):
    """torch's lazy conjugate view shares memory with unconjugated values:
    passing it must fail, not silently use the wrong sign."""
    say("fwd lazy conj view rejected")
    a = to_dev(latgen.random_lattice(64, seed=91))
    b = to_dev(latgen.random_b(seed=92))
    with pytest.raises(ValueError):
        ops.mult_nn(a.conj(), b)
    with pytest.raises(ValueError):
        ops.mult_nn(a, b.conj())
    c = ops.mult_nn(a.conj().resolve_conj(), b).cpu().numpy()
    assert np.abs(c - np.matmul(np.conj(a.cpu().numpy()), b.cpu().numpy()[None])).max() <= 1e-13
