"""GPU parity of the SoA layout: the AoS <-> SoA transforms are bit-exact
permutations (checked against the oracle's permutation and numpy's
transpose), and the SoA product matches the oracle's AoS product after the
same permutation (1e-13 in FP64, 5e-6 against the FP64 oracle in FP32)."""

import numpy as np
import pytest
import torch

import latgen
from _gpu import all_finite, say, to_dev

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
