"""GPU parity of the adjoint (su3_mult_nn_bwd) and the autograd Function.

dA: FP64 within 1e-13 max(1, max|dC|), FP32 within 5e-6 max(1, max|dC|).
dB (FP64 site sum): FP64 within 1e-12 max|dB|, FP32 within 1e-6 max|dB|,
against the oracle's compensated sum. Central differences on L = 4: the loss
is bilinear, so only rounding separates FD from the gradient (1e-6 abs).
dB is bit-identical run to run."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def _case(sites, seed=1):
    return (latgen.random_lattice(sites, seed=seed), latgen.random_b(seed=seed + 1),
            latgen.complex_normal_lattice(sites, seed=seed + 2))


@pytest.mark.parametrize("sites", [1, 7, 256, 4096, 65537])
def test_bwd_f64(O, ops, sites):
    say("bwd f64 sites=%d" % sites)
    a, b, dc = _case(sites, seed=sites)
    da, db = ops.mult_nn_bwd(to_dev(a), to_dev(b), to_dev(dc))
    da_ref, db_ref = O.mult_nn_bwd(a, b, dc)
    assert O.max_abs_diff(da.cpu().numpy(), da_ref) <= 1e-13 * max(1.0, np.abs(dc).max())
    assert O.max_abs_diff(db.cpu().numpy(), db_ref) <= 1e-12 * max(1.0, np.abs(db_ref).max())


@pytest.mark.parametrize("sites", [1, 256, 65537])
def test_bwd_f32(O, ops, sites):
    say("bwd f32 sites=%d" % sites)
    a, b, dc = _case(sites, seed=sites + 5)
    a32, b32, dc32 = O.round_f32(a), O.round_f32(b), O.round_f32(dc)
    da, db = ops.mult_nn_bwd(to_dev(a32), to_dev(b32), to_dev(dc32))
    da_ref, db_ref = O.mult_nn_bwd(a, b, dc)
    assert O.max_abs_diff(da.cpu().numpy().astype(np.complex128), da_ref) <= 5e-6 * max(1.0, np.abs(dc).max())
    assert O.max_abs_diff(db.cpu().numpy(), db_ref) <= 1e-6 * max(1.0, np.abs(db_ref).max())
    # the FP64 sum of the FP32 inputs' exact products: much tighter
    _, db_same = O.mult_nn_bwd(a32.astype(np.complex128), b32.astype(np.complex128), dc32.astype(np.complex128))
    assert O.max_abs_diff(db.cpu().numpy(), db_same) <= 1e-12 * max(1.0, np.abs(db_same).max())


def test_bwd_zero_sites(ops):
    say("bwd zero sites")
    z = torch.empty((0, 4, 3, 3), dtype=torch.complex128, device="cuda:0")
    b = to_dev(latgen.random_b())
    da, db = ops.mult_nn_bwd(z, b, z)
    assert da.shape == (0, 4, 3, 3) and torch.count_nonzero(db).item() == 0


def test_bwd_l32_and_determinism(O, ops):
    """configs: L=32 adjoint in FP64 and FP32 against the oracle; dB bitwise
    identical over 10 runs."""
    sites = 32 ** 4
    a, b, dc = _case(sites, seed=1)
    da_ref, db_ref = O.mult_nn_bwd(a, b, dc)
    for name, dt in (("f64", np.complex128), ("f32", np.complex64)):
        say("bwd L=32 %s" % name)
        ta, tb, tdc = to_dev(a.astype(dt)), to_dev(b.astype(dt)), to_dev(dc.astype(dt))
        da, db = ops.mult_nn_bwd(ta, tb, tdc)
        tol_a, tol_b = (1e-13, 1e-12) if name == "f64" else (5e-6, 1e-6)
        assert O.max_abs_diff(da.cpu().numpy().astype(np.complex128), da_ref) <= tol_a * max(1.0, np.abs(dc).max())
        assert O.max_abs_diff(db.cpu().numpy(), db_ref) <= tol_b * np.abs(db_ref).max()
        first = torch.view_as_real(db).clone()
        for _ in range(9):
            _, again = ops.mult_nn_bwd(ta, tb, tdc)
            assert torch.equal(torch.view_as_real(again), first)


def test_autograd_function_and_central_differences(O, ops):
    """SU3MultNN on L = 4 (256 sites), FP64: autograd gradients against
    central differences of the loss Re sum conj(dC) C computed with the GPU
    forward. The a-gradient uses site locality: perturbing component q of
    every site at once and reading each site's own loss term gives all 256
    site derivatives from two forward calls."""
    sites = 4 ** 4
    say("bwd autograd + FD L=4")
    a, b, dc = _case(sites, seed=77)
    ta = to_dev(a).requires_grad_(True)
    tb = to_dev(b).requires_grad_(True)
    tdc = to_dev(dc)
    c = ops.SU3MultNN.apply(ta, tb)
    loss = (torch.conj(tdc) * c).real.sum()
    loss.backward()
    ga, gb = ta.grad.cpu().numpy(), tb.grad.cpu().numpy()

    h = 1e-6
    dcn = np.conj(dc)

    def site_loss(aa, bb):
        cc = ops.mult_nn(to_dev(aa), to_dev(bb)).cpu().numpy()
        return np.sum((dcn * cc).real, axis=(1, 2, 3))

    fd_a = np.zeros_like(a)
    for j in range(4):
        for k in range(3):
            for m in range(3):
                for unit in (1.0, 1j):
                    ap = a.copy(); ap[:, j, k, m] += h * unit
                    am = a.copy(); am[:, j, k, m] -= h * unit
                    fd_a[:, j, k, m] += unit * (site_loss(ap, b) - site_loss(am, b)) / (2 * h)
    fd_b = np.zeros_like(b)
    for idx in np.ndindex(b.shape):
        for unit in (1.0, 1j):
            bp = b.copy(); bp[idx] += h * unit
            bm = b.copy(); bm[idx] -= h * unit
            fd_b[idx] += unit * (site_loss(a, bp).sum() - site_loss(a, bm).sum()) / (2 * h)
    assert O.max_abs_diff(ga, fd_a) <= 1e-6
    assert O.max_abs_diff(gb, fd_b) <= 1e-6
    da_ref, db_ref = O.mult_nn_bwd(a, b, dc)
    assert O.max_abs_diff(ga, da_ref) <= 1e-13 * max(1.0, np.abs(dc).max())
    assert O.max_abs_diff(gb, db_ref) <= 1e-12 * np.abs(db_ref).max()


def test_autograd_f32_dtype(ops):
    say("bwd autograd f32 dtype")
    a, b, dc = _case(100, seed=5)
    ta = to_dev(a.astype(np.complex64)).requires_grad_(True)
    tb = to_dev(b.astype(np.complex64)).requires_grad_(True)
    c = ops.SU3MultNN.apply(ta, tb)
    (torch.conj(to_dev(dc.astype(np.complex64))) * c).real.sum().backward()
    assert ta.grad.dtype == torch.complex64 and tb.grad.dtype == torch.complex64


def test_autograd_through_conjugate(O, ops):
    """A .conj() after the product makes autograd hand backward a lazy
    conjugate view of the upstream gradient. For L = Re sum conj(C) w, which
    equals Re sum conj(w) C, the gradients are the adjoint with dC = w."""
    say("bwd autograd through conj")
    a, b, w = _case(4099, seed=95)
    ta = to_dev(a).requires_grad_(True)
    tb = to_dev(b).requires_grad_(True)
    c = ops.SU3MultNN.apply(ta, tb)
    (c.conj() * to_dev(w)).real.sum().backward()
    da_ref, db_ref = O.mult_nn_bwd(a, b, w)
    assert O.max_abs_diff(ta.grad.cpu().numpy(), da_ref) <= 1e-13 * max(1.0, np.abs(w).max())
    assert O.max_abs_diff(tb.grad.cpu().numpy(), db_ref) <= 1e-12 * np.abs(db_ref).max()


def test_autograd_one_input(O, ops):
    """Gradients for only a, or only b, match the adjoint; the other stays None."""
    say("bwd autograd one input")
    a, b, w = _case(513, seed=97)
    da_ref, db_ref = O.mult_nn_bwd(a, b, w)
    ta = to_dev(a).requires_grad_(True)
    tb = to_dev(b)
    (torch.conj(to_dev(w)) * ops.SU3MultNN.apply(ta, tb)).real.sum().backward()
    assert O.max_abs_diff(ta.grad.cpu().numpy(), da_ref) <= 1e-13 * max(1.0, np.abs(w).max())
    assert tb.grad is None
    ta = to_dev(a)
    tb = to_dev(b).requires_grad_(True)
    (torch.conj(to_dev(w)) * ops.SU3MultNN.apply(ta, tb)).real.sum().backward()
    assert O.max_abs_diff(tb.grad.cpu().numpy(), db_ref) <= 1e-12 * np.abs(db_ref).max()
    assert ta.grad is None
