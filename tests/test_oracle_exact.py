"""Exact-arithmetic pins for the oracle's products and adjoint, over random
sizes and seeds (hypothesis). With small integer entries every FP64 product
and sum is exact, so the oracle must agree bit for bit with integer matrix
products taken through the real embedding of complex numbers, x + iy ->
[[x, -y], [y, x]], for which E(MN) = E(M) E(N) and E(M^H) = E(M)^T. A wrong
sign, a missing conjugate, a transposed operand or an index slip in any of
them changes some entry. All run on the CPU."""

import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st


def _embed(z):
    x, y = z.real.astype(np.int64), z.imag.astype(np.int64)
    blk = np.stack([np.stack([x, -y], -1), np.stack([y, x], -1)], -2)   # (..., r, c, 2, 2)
    nd = blk.ndim
    order = list(range(nd - 4)) + [nd - 4, nd - 2, nd - 3, nd - 1]
    sh = blk.shape
    return blk.transpose(order).reshape(*sh[:-4], 2 * sh[-4], 2 * sh[-3])


def _unembed(m):
    return (m[..., 0::2, 0::2] + 1j * m[..., 1::2, 0::2]).astype(np.complex128)


def _ints(rng, shape, k=9):
    return (rng.integers(-k, k + 1, size=shape) + 1j * rng.integers(-k, k + 1, size=shape)).astype(np.complex128)


def _T(m):
    return np.swapaxes(m, -1, -2)


def _same(x, y):
    return np.array_equal(x.view(np.float64), np.ascontiguousarray(y).view(np.float64))


SIZES = st.integers(min_value=1, max_value=40)
SEEDS = st.integers(min_value=0, max_value=2 ** 32 - 1)


@settings(max_examples=40, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_products_exact(O, sites, seed):
    rng = np.random.default_rng(seed)
    a, b = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3))
    A, B = _embed(a), _embed(b)[None]
    assert _same(O.mult_nn(a, b), _unembed(A @ B))
    assert _same(O.mult_na(a, b), _unembed(A @ _T(B)))
    assert _same(O.mult_an(a, b), _unembed(_T(A) @ B))
    v = _ints(rng, (sites, 3))
    V = _embed(v[:, None, :, None])[:, 0]                 # (sites, 6, 2): column vector per site
    assert _same(O.mat_vec(a, v), _unembed(A @ V[:, None])[..., 0])


@settings(max_examples=40, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_adjoint_exact(O, sites, seed):
    """dA = dC b^H per site and dB = sum_s a^H dC, both exact here (integer
    sums far below 2^53), so the compensated site sum must return the
    integer result itself."""
    rng = np.random.default_rng(seed)
    a, b, dc = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3)), _ints(rng, (sites, 4, 3, 3))
    da, db = O.mult_nn_bwd(a, b, dc)
    A, B, G = _embed(a), _embed(b)[None], _embed(dc)
    assert _same(da, _unembed(G @ _T(B)))
    assert _same(db, _unembed((_T(A) @ G).sum(axis=0)))


@settings(max_examples=30, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_form_emulators_exact(O, sites, seed):
    """The FP32, BF16 and reconstruct-12 emulators on integer entries: FP32
    arithmetic is exact here (magnitudes far below 2^24), so the FP32 and
    reconstruct-12 products equal the integer products bit for bit, and the
    BF16 product equals the integer product rounded once to BF16 (by torch,
    to nearest even)."""
    import torch
    rng = np.random.default_rng(seed)
    a, b = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3))
    A, B = _embed(a), _embed(b)[None]
    exact = _unembed(A @ B)
    b32 = b.astype(np.complex64)
    c32 = O.mult_nn_f32(a.astype(np.complex64), b32)
    assert np.array_equal(c32.view(np.float32), exact.astype(np.complex64).view(np.float32))
    c16 = O.mult_nn_bf16(O.round_bf16(a), b32)                              # uint16 (..., 2)
    want16 = torch.from_numpy(exact.view(np.float64).reshape(c16.shape)).to(torch.float32).to(torch.bfloat16)
    assert np.array_equal(c16.view(np.int16), want16.view(torch.int16).numpy())
    r0, r1 = a[..., 0, :], a[..., 1, :]
    row2 = np.conj(np.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                             r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                             r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], -1))
    a12 = a.copy()
    a12[:, :, 2, :] = row2
    c12 = O.mult_nn_r12(O.pack_r12(a), b32)
    assert np.array_equal(c12.view(np.float32), _unembed(_embed(a12) @ B).astype(np.complex64).view(np.float32))
