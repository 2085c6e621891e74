"""Seeded input generator: determinism, independence from chunking, and the
distributional facts the workloads rely on."""

import numpy as np

import latgen


def test_splitmix64_reference_sequence():
    """SplitMix64 from state 0 yields the published sequence
    e220a8397b1dcdaf, 6e789e6aa1b965f4, 06c45d188009454f."""
    g = 0x9E3779B97F4A7C15
    out = [latgen._splitmix64_scalar((i * g) % 2 ** 64) for i in range(3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = latgen._splitmix64(np.array([0, g, (2 * g) % 2 ** 64], dtype=np.uint64))
    assert [int(x) for x in v] == out


def test_uniform_open_interval_and_moments():
    u = latgen.uniform(9, np.arange(1 << 20, dtype=np.uint64))
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 2e-3
    assert abs(u.var() - 1 / 12) < 2e-3


def test_values_independent_of_chunking(monkeypatch):
    ref = latgen.haar_su3(5, 0, 5000)
    monkeypatch.setattr(latgen, "_CHUNK", 777)
    again = latgen.haar_su3(5, 0, 5000)
    assert np.array_equal(ref, again)
    # an offset window equals the slice of the full run
    assert np.array_equal(latgen.haar_su3(5, 1234, 100), ref[1234:1334])
    # lattice: matrix m = 4 s + j
    lat = latgen.random_lattice(1250, seed=5)
    assert np.array_equal(lat.reshape(-1, 3, 3), ref)


def test_haar_su3_properties():
    u = latgen.haar_su3(1, 0, 200000)
    uh = np.conj(np.swapaxes(u, 1, 2))
    dev = np.abs(np.matmul(uh, u) - np.eye(3)).max()
    assert dev < 5e-15
    d = np.linalg.det(u)
    assert np.abs(d - 1).max() < 5e-15
    # Haar: each |U_kl|^2 has mean 1/3 and E|U_00|^4 = 1/6 (Beta(1, 2))
    p = np.abs(u) ** 2
    assert np.abs(p.mean(axis=0) - 1 / 3).max() < 3e-3
    assert abs((p[:, 0, 0] ** 2).mean() - 1 / 6) < 3e-3
    # no preferred phase
    assert abs(u[:, 1, 2].mean()) < 5e-3


def test_complex_normal_moments():
    z = latgen.complex_normal_lattice(1 << 14, seed=3).ravel()
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 1e-2
    assert abs(z.real.var() - 0.5) < 1e-2 and abs(z.imag.var() - 0.5) < 1e-2
    assert abs(np.mean(z * z)) < 1e-2          # circular


def test_structured_inputs():
    b = latgen.permutation_b()
    for m in b:
        assert np.allclose(m.conj().T @ m, np.eye(3)) and abs(np.linalg.det(m) - 1) < 1e-15
    assert not np.array_equal(b[1], b[1].T)
    q = latgen.index_coded(10)
    assert q[3, 2, 1, 0] == (((3 * 4 + 2) * 3 + 1) * 3 + 0) - 1j * ((((3 * 4 + 2) * 3 + 1) * 3) + 0.5)
    a, bb = latgen.paper_init(3)
    assert np.all(a == 1) and np.all(bb == 1.0 / 3.0)
