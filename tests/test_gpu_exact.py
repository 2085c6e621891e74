"""Exact-arithmetic GPU parity. With integer entries in [-9, 9] every
operation the kernels perform is exact: FP64 and FP32 products and sums
(magnitudes far below 2^24), the BF16 form's FP32 product before its final
rounding, the rebuilt third row of the reconstruct-12 forms, and the FP64
site sum of dB. So every result must equal exact integer arithmetic bit for
bit: integer matrix products through the real embedding x + iy ->
[[x, -y], [y, x]] (numpy int64), rounded to BF16 by torch where the form
stores BF16. Sizes are drawn at random (hypothesis), ragged included."""

import numpy as np
import pytest
import torch
from hypothesis import given, settings
from hypothesis import strategies as st

from _gpu import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_2103_00571_amd import ops
    return ops


def _embed(z):
    """Entry (k, l) = x + iy becomes the 2x2 block [[x, -y], [y, x]] at rows
    2k, 2k+1 and columns 2l, 2l+1 (int64)."""
    x, y = np.rint(z.real).astype(np.int64), np.rint(z.imag).astype(np.int64)
    out = np.empty(z.shape[:-2] + (2 * z.shape[-2], 2 * z.shape[-1]), dtype=np.int64)
    out[..., 0::2, 0::2] = x
    out[..., 0::2, 1::2] = -y
    out[..., 1::2, 0::2] = y
    out[..., 1::2, 1::2] = x
    return out


def _unembed(m):
    return (m[..., 0::2, 0::2] + 1j * m[..., 1::2, 0::2]).astype(np.complex128)


def _T(m):
    return np.swapaxes(m, -1, -2)


def _ints(rng, shape):
    return (rng.integers(-9, 10, size=shape) + 1j * rng.integers(-9, 10, size=shape)).astype(np.complex128)


def _cross_row2(a):
    """conj(row0 x row1) per link, in exact integers."""
    r0, r1 = a[..., 0, :], a[..., 1, :]
    x = np.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                  r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                  r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], -1)
    return np.conj(x)


def _same(got, want):
    got = got.detach().cpu()
    want = torch.from_numpy(np.ascontiguousarray(want)).to(got.dtype)
    return torch.equal(torch.view_as_real(got), torch.view_as_real(want))


def _bf16_same(got, want):
    if isinstance(want, torch.Tensor):
        want = want.cpu().numpy()
    want = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(want))).to(torch.float32).to(torch.bfloat16)
    return torch.equal(got.cpu().view(torch.int16), want.view(torch.int16))


SIZES = st.one_of(st.sampled_from([1, 2, 3, 63, 64, 65, 4097]), st.integers(min_value=1, max_value=70000))
SEEDS = st.integers(min_value=0, max_value=2 ** 32 - 1)


@settings(max_examples=12, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_forward_forms_exact(ops, sites, seed):
    say("exact forward forms sites=%d seed=%d" % (sites, seed))
    rng = np.random.default_rng(seed)
    a, b = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3))
    A, B = _embed(a), _embed(b)[None]
    want = _unembed(A @ B)
    ta, tb = to_dev(a), to_dev(b)
    tb32 = tb.to(torch.complex64)
    assert _same(ops.mult_nn(ta, tb), want)
    assert _same(ops.mult_nn(ops.pack(ta, ops.SU3_F32), tb32), want)
    assert _bf16_same(ops.mult_nn(ops.pack(ta, ops.SU3_BF16), tb32), want)
    assert _same(ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(ta), tb)), want)
    # reconstruct-12: the kernels rebuild row 2 as conj(row0 x row1)
    a12 = a.copy()
    a12[:, :, 2, :] = _cross_row2(a)
    want12 = _unembed(_embed(a12) @ B)
    assert _same(ops.mult_nn(ops.pack(ta, ops.SU3_R12_F32), tb32), want12)
    assert _same(ops.mult_nn(ops.pack(ta, ops.SU3_R12_F64), tb), want12)
    assert _same(ops.mult_nn(ops.pack(ta, ops.SU3_R12C_F32), tb32, form=ops.SU3_R12C_F32), want[:, :, :2, :])


@settings(max_examples=12, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_other_products_exact(ops, sites, seed):
    say("exact a b^H, a^H b, matrix x vector sites=%d seed=%d" % (sites, seed))
    rng = np.random.default_rng(seed)
    a, b, v = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3)), _ints(rng, (sites, 3))
    A, B = _embed(a), _embed(b)[None]
    V = _embed(v[:, None, :, None])[:, 0]
    for dt in (torch.complex128, torch.complex64):
        ta, tb, tv = to_dev(a).to(dt), to_dev(b).to(dt), to_dev(v).to(dt)
        assert _same(ops.mult_na(ta, tb), _unembed(A @ _T(B)))
        assert _same(ops.mult_an(ta, tb), _unembed(_T(A) @ B))
        assert _same(ops.mat_vec(ta, tv), _unembed(A @ V[:, None])[..., 0])


@settings(max_examples=12, deadline=None)
@given(sites=SIZES, seed=SEEDS)
def test_adjoint_exact(ops, sites, seed):
    say("exact adjoint sites=%d seed=%d" % (sites, seed))
    rng = np.random.default_rng(seed)
    a, b, dc = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3)), _ints(rng, (sites, 4, 3, 3))
    A, B, G = _embed(a), _embed(b)[None], _embed(dc)
    want_da = _unembed(G @ _T(B))
    want_db = _unembed((_T(A) @ G).sum(axis=0))
    for dt in (torch.complex128, torch.complex64):
        da, db = ops.mult_nn_bwd(to_dev(a).to(dt), to_dev(b).to(dt), to_dev(dc).to(dt))
        assert _same(da, want_da)
        assert _same(db, want_db)


def test_beyond_2_31_chunks(ops):
    """A lattice of 60,000,000 sites (FP64: 2.16e9 16-byte chunks, 34.6 GB
    per array), past the range of 32-bit chunk indices: the site-major
    product, the SoA product and a b^H on integer entries, bit-exact on
    20,000 sampled sites plus the first and last 64."""
    sites = 60_000_000
    assert sites * 36 > 2 ** 31
    say("exact sites=%d (beyond 2^31 chunks)" % sites)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(2031)
    a = torch.view_as_complex(torch.randint(-9, 10, (sites, 4, 3, 3, 2), generator=g, device=dev,
                                            dtype=torch.float64))
    rng = np.random.default_rng(2031)
    b = _ints(rng, (4, 3, 3))
    tb = to_dev(b)
    idx = np.unique(np.concatenate([rng.integers(0, sites, 20000), np.arange(64), np.arange(sites - 64, sites)]))
    tidx = torch.from_numpy(idx).to(dev)
    A, B = _embed(a[tidx].cpu().numpy()), _embed(b)[None]
    want = _unembed(A @ B)
    c = ops.mult_nn(a, tb)
    assert _same(c[tidx], want)
    say("  a b^H")
    ops.mult_na(a, tb, out=c)
    assert _same(c[tidx], _unembed(A @ _T(B)))
    del c
    say("  SoA")
    sa = ops.aos_to_soa(a)
    del a
    sc = ops.mult_nn_soa(sa, tb)
    del sa
    assert _same(ops.soa_to_aos(sc)[tidx], want)


def _grid_sizes(scale):
    """Site counts whose tile counts (one workgroup per tile) take every
    residue mod 8 for every kernel that deals tiles out XCD-contiguously:
    16k+5 sites give ceil(s/16) = k+1 and ceil(3s/16) = 3k+1, 32k+7 give
    ceil(s/32) = k+1 and ceil(3s/32) = 3k+1, 64k+11 give ceil(3s/64) = 3k+1,
    over 8 consecutive k. `scale` (a multiple of 8) is added to k."""
    return [m * (k + scale) + r for m, r in ((16, 5), (32, 7), (64, 11)) for k in range(8, 16)]


def _check_all_products(ops, a, b, v, want, want12, want_na, want_an, want_mv, same):
    """Every product and the reconstruct-12 pack and unpack against exact
    expected values; same(got, want) compares bit for bit."""
    tb32, tv32 = b.to(torch.complex64), v.to(torch.complex64)
    assert same(ops.mult_nn(a, b), want)
    assert same(ops.mult_nn(ops.pack(a, ops.SU3_F32), tb32), want)
    assert _bf16_same(ops.mult_nn(ops.pack(a, ops.SU3_BF16), tb32), want)
    p12, p12d = ops.pack(a, ops.SU3_R12_F32), ops.pack(a, ops.SU3_R12_F64)
    assert same(p12, want12[:, :, :2, :]) and same(p12d, want12[:, :, :2, :])
    assert same(ops.unpack(p12, ops.SU3_R12_F32), want12) and same(ops.unpack(p12d, ops.SU3_R12_F64), want12)
    assert same(ops.mult_nn(ops.pack(a, ops.SU3_R12C_F32), tb32, form=ops.SU3_R12C_F32), want[:, :, :2, :])
    for x, y, w in ((a, b, v), (a.to(torch.complex64), tb32, tv32)):
        assert same(ops.mult_na(x, y), want_na)
        assert same(ops.mult_an(x, y), want_an)
        assert same(ops.mat_vec(x, w), want_mv)


def test_every_grid_residue_exact(ops):
    """The XCD-contiguous tile order maps workgroups onto tiles one to one for
    every grid size: each product and the reconstruct-12 pack and unpack, on
    grids of every residue mod 8, bit-exact against integer arithmetic, with
    the workgroup counts checked."""
    rng = np.random.default_rng(808)
    seen = set()
    for sites in _grid_sizes(0):
        say("exact grid residues sites=%d" % sites)
        grid, _ = ops.launch_shape(sites, ops.SU3_F64)
        assert grid == -(-12 * sites // 64)
        seen.add(grid % 8)
        a, b, v = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3)), _ints(rng, (sites, 3))
        A, B = _embed(a), _embed(b)[None]
        V = _embed(v[:, None, :, None])[:, 0]
        a12 = a.copy()
        a12[:, :, 2, :] = _cross_row2(a)
        # products whose results are written on the rebuilt links compare
        # against a12 (the stored rows 0-1 and the rebuilt row 2)
        _check_all_products(ops, to_dev(a), to_dev(b), to_dev(v), _unembed(A @ B), a12,
                            _unembed(A @ _T(B)), _unembed(_T(A) @ B), _unembed(A @ V[:, None])[..., 0], _same)
        w12 = _unembed(_embed(a12) @ B)
        assert _same(ops.mult_nn(ops.pack(to_dev(a), ops.SU3_R12_F32), to_dev(b).to(torch.complex64)), w12)
        assert _same(ops.mult_nn(ops.pack(to_dev(a), ops.SU3_R12_F64), to_dev(b)), w12)
    assert seen == set(range(8))


def test_every_grid_residue_exact_large(ops):
    """The same on grids about 24,000 (FP64 forward) to 8,000 (reconstruct-12)
    tiles long, every residue mod 8 again. The expected values come from
    torch's complex128 products on the GPU, exact for these integer entries
    (every partial sum is an integer far below 2^53)."""
    rng = np.random.default_rng(809)
    seen = set()
    for sites in _grid_sizes(8000)[:16]:
        say("exact grid residues sites=%d" % sites)
        grid, _ = ops.launch_shape(sites, ops.SU3_F64)
        seen.add(grid % 8)
        a, b, v = (to_dev(_ints(rng, sh)) for sh in ((sites, 4, 3, 3), (4, 3, 3), (sites, 3)))
        bh = b.conj().transpose(-1, -2).resolve_conj().contiguous()
        ah = a.conj().transpose(-1, -2).resolve_conj().contiguous()
        r0, r1 = a[:, :, 0, :], a[:, :, 1, :]
        a12 = a.clone()
        for p, (i, j) in enumerate(((1, 2), (2, 0), (0, 1))):
            a12[:, :, 2, p] = torch.conj(r0[..., i] * r1[..., j] - r0[..., j] * r1[..., i])
        want, want_mv = torch.matmul(a, b), torch.matmul(a, v[:, None, :, None])[..., 0]

        def same(got, w):
            return torch.equal(torch.view_as_real(got.to(torch.complex128)), torch.view_as_real(w))
        _check_all_products(ops, a, b, v, want, a12, torch.matmul(a, bh), torch.matmul(ah, b), want_mv, same)
        w12 = torch.matmul(a12, b)
        assert same(ops.mult_nn(ops.pack(a, ops.SU3_R12_F32), b.to(torch.complex64)), w12)
        assert same(ops.mult_nn(ops.pack(a, ops.SU3_R12_F64), b), w12)
    assert seen == set(range(8))


def test_soa_xcd_order_every_residue_exact(ops):
    """The FP64 SoA product deals a row's site blocks out XCD-contiguously
    when the plane stride (16 B x sites) lies within 128 KiB of a multiple of
    4 MiB, padding the row's workgroup count to a multiple of 8. Site counts
    2^18 + 128 k (+ 37) pick that order, with block counts of every residue
    mod 8, ragged or not; every output must equal integer arithmetic, in
    FP64 and (tile = workgroup index) FP32."""
    rng = np.random.default_rng(818)
    seen = set()
    for k in range(8):
        for r in (0, 37):
            sites = 2 ** 18 + 128 * k + r
            m = (16 * sites) % (4 << 20)
            assert m < (128 << 10) or m > (4 << 20) - (128 << 10)
            seen.add(-(-sites // 128) % 8)
            say("exact SoA XCD order sites=%d" % sites)
            a, b = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3))
            want = _unembed(_embed(a) @ _embed(b)[None])
            ta, tb = to_dev(a), to_dev(b)
            for dt in (torch.complex128, torch.complex64):
                sa = ops.aos_to_soa(ta.to(dt))
                assert _same(ops.soa_to_aos(ops.mult_nn_soa(sa, tb.to(dt))), want)
    assert seen == set(range(8))


def test_soa_pitched_exact(ops):
    """The padded SoA layout at site counts whose dense plane stride aliases
    in HBM (2^20, 2^20 - 64, 2^18 + 37) and at a small ragged one, each at
    the recommended pitch and at that pitch + 37 (odd): every output equals
    integer arithmetic bit for bit in FP64 and FP32."""
    rng = np.random.default_rng(919)
    for sites in (2 ** 20, 2 ** 20 - 64, 2 ** 18 + 37, 999):
        a, b = _ints(rng, (sites, 4, 3, 3)), _ints(rng, (4, 3, 3))
        want = _unembed(_embed(a) @ _embed(b)[None])
        ta, tb = to_dev(a), to_dev(b)
        for dt, form in ((torch.complex128, ops.SU3_F64), (torch.complex64, ops.SU3_F32)):
            p0 = ops.soa_pitch(sites, form)
            for pitch in (p0, p0 + 37):
                say("exact SoA pitched sites=%d pitch=%d form=%d" % (sites, pitch, form))
                sa = ops.aos_to_soa(ta.to(dt), pitch)
                sc = ops.mult_nn_soa(sa, tb.to(dt), sites=sites)
                assert _same(ops.soa_to_aos(sc, sites), want)


def test_soa_load_phases_exact(ops):
    """The SoA product on the dense layout splits each thread's three plane
    loads into phases, from the plane stride S: FP32 waits before plane 2,
    and after every plane where S lies within 128 KiB of a multiple of 8 MiB
    and is at least 16 MiB; FP64 waits after plane 0 where S lies within
    128 KiB of a multiple of 16 MiB (and is at least 16 MiB), else not at
    all. Site counts that take each choice, ragged ones among them, and the
    padded layout (no waits), must equal integer arithmetic bit for bit. The
    expected products are torch's complex128 products on the GPU, exact for
    these integer entries."""
    rng = np.random.default_rng(919191)

    def near(stride, period):
        m = stride % period
        return m < (128 << 10) or m > period - (128 << 10)

    lo16 = (16 << 20) - (128 << 10)
    cases = ((ops.SU3_F32, 999, 1), (ops.SU3_F32, 2 ** 20, 1), (ops.SU3_F32, 2 ** 21 + 37, 2),
             (ops.SU3_F32, 3 * 2 ** 20 + 5000, 2), (ops.SU3_F64, 999, 0), (ops.SU3_F64, 2 ** 19, 0),
             (ops.SU3_F64, 2 ** 20, 1), (ops.SU3_F64, 2 ** 20 + 37, 1), (ops.SU3_F64, 3 * 2 ** 20 - 3000, 1))
    for form, sites, waits in cases:
        es = 16 if form == ops.SU3_F64 else 8
        stride = es * sites
        if form == ops.SU3_F64:
            assert waits == (1 if stride >= lo16 and near(stride, 16 << 20) else 0)
        else:
            assert waits == (2 if near(stride, 8 << 20) and stride >= lo16 else 1)
        say("exact SoA load phases form=%d sites=%d waits=%d" % (form, sites, waits))
        a = to_dev(_ints(rng, (sites, 4, 3, 3)))
        b = to_dev(_ints(rng, (4, 3, 3)))
        want = torch.matmul(a, b)
        dt = torch.complex128 if form == ops.SU3_F64 else torch.complex64
        ax, bx = a.to(dt), b.to(dt)
        got = ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(ax), bx))
        assert torch.equal(torch.view_as_real(got.to(torch.complex128)), torch.view_as_real(want))
        pitch = ops.soa_pitch(sites, form)
        got = ops.soa_to_aos(ops.mult_nn_soa(ops.aos_to_soa(ax, pitch), bx, sites=sites), sites)
        assert torch.equal(torch.view_as_real(got.to(torch.complex128)), torch.view_as_real(want))
        del a, ax, want, got
