"""Pins for the oracle: checks of `oracle/` against what the paper and the
mathematics fix, never against the oracle's own formulas.

Each test names the plausible oracle mistake it would catch. All run on the
CPU.
"""

import math
import os

import numpy as np
import pytest
import torch

import latgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _ulp(x):
    return np.spacing(np.abs(x).astype(np.float64))


# --------------------------------------------------------------- forward O1

def test_identity_b_returns_a_exactly(O):
    """P1: b[j] = I gives c == a bit for bit (catches a wrong link or row index,
    a dropped or extra term: any of them changes some entry)."""
    a = latgen.random_lattice(256, seed=11)
    c = O.mult_nn(a, latgen.identity_b())
    assert np.array_equal(c.view(np.float64), a.view(np.float64))


def test_signed_permutation_b_is_exact_column_permutation(O):
    """P2: b = (I, P, P^2, diag(i, i, -1)) moves columns of a.

    c[s][1][k][l] = a[s][1][k][(l+1)%3], c[s][2][k][l] = a[s][2][k][(l+2)%3],
    c[s][3] = a[s][3] * (i, i, -1) by column. Catches b used transposed (P^T =
    P^2 would swap links 1 and 2), a wrong j, and a wrong sign of the
    imaginary part of the product (the factor i)."""
    a = latgen.random_lattice(300, seed=12)
    c = O.mult_nn(a, latgen.permutation_b())
    assert np.array_equal(c[:, 0], a[:, 0])
    for l in range(3):
        assert np.array_equal(c[:, 1, :, l], a[:, 1, :, (l + 1) % 3])
        assert np.array_equal(c[:, 2, :, l], a[:, 2, :, (l + 2) % 3])
    # multiplying by i: (x + iy) i = -y + ix, exact
    for l in range(2):
        assert np.array_equal(c[:, 3, :, l].real, -a[:, 3, :, l].imag)
        assert np.array_equal(c[:, 3, :, l].imag, a[:, 3, :, l].real)
    assert np.array_equal(c[:, 3, :, 2], -a[:, 3, :, 2])


def test_paper_initialisation_gives_exact_one(O):
    """P3: the paper's own init (a = 1, b = 1/3) gives c = 1 + 0i exactly,
    in FP64 and in the FP32 form; values read from the golden fixture."""
    g = _golden("paper_init.txt")
    sites = 1000
    a = np.full((sites, 4, 3, 3), complex(g["a_re"], g["a_im"]))
    b = np.full((4, 3, 3), complex(g["b_numerator"] / g["b_denominator"], 0.0))
    a2, b2 = latgen.paper_init(sites)
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    c = O.mult_nn(a, b)
    assert np.all(c.real == g["c_re"]) and np.all(c.imag == g["c_im"])
    c32 = O.mult_nn_f32(a.astype(np.complex64), b.astype(np.complex64))
    assert np.all(c32.real == np.float32(g["c_re"])) and np.all(c32.imag == 0)


def test_against_numpy_matmul(O):
    """P4: a library routine (numpy matmul over the stacked links)."""
    a = latgen.random_lattice(4096, seed=1)
    b = latgen.random_b(seed=2)
    c = O.mult_nn(a, b)
    ref = np.matmul(a, b[None])
    assert O.max_abs_diff(c, ref) <= 1e-15


def test_exact_integer_product_by_real_embedding(O):
    """P5: brute force with exact integers. A complex x + iy is the real 2x2
    block [[x, -y], [y, x]]; a 3x3 complex link is then a 6x6 integer matrix
    and the integer matmul is exact. Small integer entries make every FP64
    product and sum exact, so the oracle must agree bit for bit. Catches a
    wrong sign in either part of the complex product and any index slip."""
    rng = np.random.default_rng(5)
    sites = 16  # a 2^4 lattice
    ar = rng.integers(-8, 9, size=(sites, 4, 3, 3, 2))
    br = rng.integers(-8, 9, size=(4, 3, 3, 2))

    def embed(z):
        x, y = z[..., 0], z[..., 1]
        top = np.stack([x, -y], axis=-1)
        bot = np.stack([y, x], axis=-1)
        blk = np.stack([top, bot], axis=-2)              # (..., 3, 3, 2, 2)
        sh = blk.shape[:-4]
        return blk.transpose(*range(len(sh)), -4, -2, -3, -1).reshape(*sh, 6, 6)

    A6, B6 = embed(ar), embed(br)
    C6 = np.matmul(A6, B6[None])                          # int64, exact
    cre = C6[..., 0::2, 0::2]
    cim = C6[..., 1::2, 0::2]
    a = ar[..., 0] + 1j * ar[..., 1]
    b = br[..., 0] + 1j * br[..., 1]
    c = O.mult_nn(a, b)
    assert np.array_equal(c.real, cre.astype(np.float64))
    assert np.array_equal(c.imag, cim.astype(np.float64))


def test_su3_closure(O):
    """P6: products of SU(3) matrices stay in SU(3) (group closure):
    ||C^H C - I||_F <= 1e-13 and |det C - 1| <= 1e-13."""
    a = latgen.random_lattice(8 ** 4, seed=1)
    b = latgen.random_b(seed=2)
    c = O.mult_nn(a, b)
    assert O.unitarity_dev(c) <= 1e-13
    assert O.det_dev(c) <= 1e-13


def test_linearity_and_associativity(O):
    """P7: c is linear in a, and (a b1) b2 = a (b1 b2)."""
    a1 = latgen.random_lattice(512, seed=21)
    a2 = latgen.random_lattice(512, seed=22)
    b1 = latgen.random_b(seed=23)
    b2 = latgen.random_b(seed=24)
    alpha = 0.37 - 1.25j
    lhs = O.mult_nn(alpha * a1 + a2, b1)
    rhs = alpha * O.mult_nn(a1, b1) + O.mult_nn(a2, b1)
    assert O.max_abs_diff(lhs, rhs) <= 1e-14
    b12 = np.matmul(b1, b2)
    assert O.max_abs_diff(O.mult_nn(O.mult_nn(a1, b1), b2), O.mult_nn(a1, b12)) <= 1e-14


def test_site_locality(O):
    """P12: changing a[s] changes c[s] only."""
    a = latgen.random_lattice(64, seed=31)
    b = latgen.random_b(seed=32)
    c0 = O.mult_nn(a, b)
    a[17, 2, 1, 0] += 0.5
    c1 = O.mult_nn(a, b)
    diff = np.any(c0 != c1, axis=(1, 2, 3))
    assert diff[17] and diff.sum() == 1
    # within the site only link 2, row 1 changes
    d = c0[17] != c1[17]
    assert d[2, 1].all() and d.sum() == 3


def test_empty_lattice(O):
    a = np.zeros((0, 4, 3, 3), dtype=np.complex128)
    c = O.mult_nn(a, latgen.random_b())
    assert c.shape == (0, 4, 3, 3)


# --------------------------------------------------------------- adjoint O2

def test_adjoint_against_torch_autograd(O):
    """P10: torch autograd of torch.matmul on complex128 (CPU) for the loss
    Re sum conj(dC) * C; uses the same complex-gradient convention."""
    sites = 16
    a = latgen.random_lattice(sites, seed=41)
    b = latgen.random_b(seed=42)
    dc = latgen.complex_normal_lattice(sites, seed=43)
    ta = torch.tensor(a, requires_grad=True)
    tb = torch.tensor(b, requires_grad=True)
    tc = torch.matmul(ta, tb.unsqueeze(0))
    loss = (torch.conj(torch.tensor(dc)) * tc).real.sum()
    loss.backward()
    da, db = O.mult_nn_bwd(a, b, dc)
    assert O.max_abs_diff(da, ta.grad.numpy()) <= 1e-14
    assert O.max_abs_diff(db, tb.grad.numpy()) <= 1e-13


def test_adjoint_against_central_differences(O):
    """P10: central finite differences of the loss Re sum conj(dC) * C built
    on the oracle's forward. The loss is bilinear in (a, b), so the central
    difference has no truncation error; only rounding remains (h = 1e-6)."""
    sites = 4
    a = latgen.random_lattice(sites, seed=51)
    b = latgen.random_b(seed=52)
    dc = latgen.complex_normal_lattice(sites, seed=53)
    h = 1e-6

    def loss(aa, bb):
        return float(np.sum((np.conj(dc) * O.mult_nn(aa, bb)).real))

    da, db = O.mult_nn_bwd(a, b, dc)
    fd_a = np.zeros_like(a)
    for idx in np.ndindex(a.shape):
        for part, unit in ((0, 1.0), (1, 1j)):
            ap = a.copy(); ap[idx] += h * unit
            am = a.copy(); am[idx] -= h * unit
            g = (loss(ap, b) - loss(am, b)) / (2 * h)
            if part == 0:
                fd_a[idx] += g
            else:
                fd_a[idx] += 1j * g
    fd_b = np.zeros_like(b)
    for idx in np.ndindex(b.shape):
        for part, unit in ((0, 1.0), (1, 1j)):
            bp = b.copy(); bp[idx] += h * unit
            bm = b.copy(); bm[idx] -= h * unit
            g = (loss(a, bp) - loss(a, bm)) / (2 * h)
            fd_b[idx] += g if part == 0 else 1j * g
    assert O.max_abs_diff(da, fd_a) <= 1e-6
    assert O.max_abs_diff(db, fd_b) <= 1e-6


def test_adjoint_db_is_correctly_rounded_sum(O):
    """The oracle's dB equals math.fsum (an exactly rounded sum, Shewchuk)
    of the same rounded terms to within 1 ulp. Catches a missing
    compensation or a dropped site."""
    sites = 256
    a = latgen.random_lattice(sites, seed=61)
    b = latgen.random_b(seed=62)
    dc = latgen.complex_normal_lattice(sites, seed=63)
    _, db = O.mult_nn_bwd(a, b, dc)
    ar, ai = a.real, -a.imag
    gr, gi = dc.real, dc.imag
    for j in range(4):
        for m in range(3):
            for l in range(3):
                x1 = np.multiply(ar[:, j, :, m], gr[:, j, :, l])
                x2 = np.multiply(ai[:, j, :, m], gi[:, j, :, l])
                y1 = np.multiply(ar[:, j, :, m], gi[:, j, :, l])
                y2 = np.multiply(ai[:, j, :, m], gr[:, j, :, l])
                re = math.fsum(np.subtract(x1, x2).ravel())
                im = math.fsum(np.add(y1, y2).ravel())
                assert abs(db[j, m, l].real - re) <= _ulp(re)
                assert abs(db[j, m, l].imag - im) <= _ulp(im)


# ------------------------------------------------------------ recon-12 (O3)

def test_recon_matches_independent_third_row(O):
    """P8: the generator builds row 2 by Gram-Schmidt and a determinant phase,
    never by a cross product; the oracle's conj(r0 x r1) must reproduce it."""
    a = latgen.random_lattice(512, seed=71).reshape(-1, 3, 3)
    worst = 0.0
    for u in a[:400]:
        worst = max(worst, np.abs(O.recon_row2(u[0], u[1]) - u[2]).max())
    assert worst <= 1e-14


def test_recon_reversed_order_has_det_minus_one(O):
    """Negative test: conj(r1 x r0) (reversed cross order) gives det = -1, so
    a swapped cross product cannot pass the det = 1 check."""
    u = latgen.haar_su3(72, 0, 8)
    for m in u:
        wrong = np.stack([m[0], m[1], O.recon_row2(m[1], m[0])])
        right = np.stack([m[0], m[1], O.recon_row2(m[0], m[1])])
        assert abs(O.det(wrong) + 1) <= 1e-14
        assert abs(O.det(right) - 1) <= 1e-14


def test_pack_unpack_r12(O):
    """pack keeps rows 0-1 rounded to FP32 (bit-exact vs numpy's RNE cast);
    unpack widens them exactly and rebuilds row 2 within FP32 input error."""
    a = latgen.random_lattice(300, seed=73)
    p = O.pack_r12(a)
    assert np.array_equal(p.view(np.float32), a[:, :, :2, :].astype(np.complex64).view(np.float32))
    u = O.unpack_r12(p)
    assert np.array_equal(u[:, :, :2, :], p.astype(np.complex128))
    assert O.max_abs_diff(u, a) <= 1e-6
    assert O.det_dev(u) <= 1e-6


# -------------------------------------------------------------- metrics (O4)

def test_metrics_closed_forms(O):
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), (5, 3, 3)).copy()
    assert O.unitarity_dev(eye) == 0.0 and O.det_dev(eye) == 0.0
    # M = 2I: M^H M - I = 3I, Frobenius norm 3*sqrt(3); det = 8
    assert O.unitarity_dev(2 * eye) == pytest.approx(3 * math.sqrt(3), rel=1e-15)
    assert O.det_dev(2 * eye) == pytest.approx(7.0, rel=1e-15)
    # a diagonal phase matrix is unitary
    ph = np.diag(np.exp(1j * np.array([0.3, -1.1, 2.0])))
    assert O.unitarity_dev(ph[None]) <= 1e-15
    assert O.det(np.diag([2.0, 3.0j, 5.0])) == 30j
    rng = np.random.default_rng(3)
    for _ in range(20):
        m = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
        assert abs(O.det(m) - np.linalg.det(m)) <= 1e-13
    x = np.array([1.0, -2.0, 3.0])
    y = np.array([1.5, -2.0, 0.0])
    assert O.max_abs_diff(x, y) == 3.0
    assert O.max_abs_diff(np.array([np.nan]), np.array([0.0])) == math.inf


# ---------------------------------------------------------- storage forms (O5)

def test_round_f32_matches_numpy_rne(O):
    a = latgen.random_lattice(256, seed=81)
    assert np.array_equal(O.round_f32(a).view(np.float32), a.astype(np.complex64).view(np.float32))


def _bf16_torch(x):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def test_bf16_rounding_matches_torch_and_ties_to_even(O):
    """FP32 -> BF16 is bit-exact against torch's CPU conversion, including
    exact ties; FP64 -> BF16 goes through FP32 (A10)."""
    rng = np.random.default_rng(7)
    x = rng.normal(size=100000).astype(np.float32)
    # exact ties: low 16 bits 0x8000, both parities of bit 16
    bits = rng.integers(0, 1 << 31, size=4096, dtype=np.uint32)
    ties = ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32)
    ties = ties[np.isfinite(ties)]
    for v in (x, ties, np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 1e-40], dtype=np.float32)):
        assert np.array_equal(O.f32_to_bf16(v), _bf16_torch(v))
    # hand-checked ties: 1 + 2^-8 -> 1.0 (0x3F80); 1 + 3*2^-8 -> 1 + 2^-6 (0x3F82)
    assert O.f32_to_bf16(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8], dtype=np.float32)).tolist() == [0x3F80, 0x3F82]
    d = rng.normal(size=(1000, 4, 3, 3)) + 1j * rng.normal(size=(1000, 4, 3, 3))
    h = O.round_bf16(d)
    assert np.array_equal(h, _bf16_torch(d.astype(np.complex64).view(np.float32)).reshape(h.shape))
    w = O.widen_bf16(h)
    assert np.array_equal(w.view(np.float64).reshape(-1),
                          h.reshape(-1).astype(np.uint32).__lshift__(16).view(np.float32).astype(np.float64))


def test_f32_form_emulator(O):
    """FP32 emulator: exact pins P1-P3 and a library cross-check."""
    a = latgen.random_lattice(1024, seed=91)
    a32 = O.round_f32(a)
    c_id = O.mult_nn_f32(a32, latgen.identity_b().astype(np.complex64))
    assert np.array_equal(c_id.view(np.float32), a32.view(np.float32))
    c_p = O.mult_nn_f32(a32, latgen.permutation_b().astype(np.complex64))
    for l in range(3):
        assert np.array_equal(c_p[:, 1, :, l], a32[:, 1, :, (l + 1) % 3])
    b32 = O.round_f32(latgen.random_b(seed=92))
    c = O.mult_nn_f32(a32, b32)
    ref = np.matmul(a32.astype(np.complex128), b32.astype(np.complex128)[None])
    assert O.max_abs_diff(c.astype(np.complex128), ref) <= 1e-6
    # and against the FP64 definition on the unrounded inputs (tolerance 5e-6)
    c64 = O.mult_nn(a, latgen.random_b(seed=92))
    assert O.max_abs_diff(c.astype(np.complex128), c64) <= 5e-6


def test_bf16_form_emulator(O):
    """BF16 emulator: b = I returns a bit for bit; paper init gives exact 1;
    random SU(3) stays within one BF16 ulp of the rounded FP64 product."""
    a = latgen.random_lattice(1024, seed=101)
    a16 = O.round_bf16(a)
    eye32 = latgen.identity_b().astype(np.complex64)
    assert np.array_equal(O.mult_nn_bf16(a16, eye32), a16)
    pa, pb = latgen.paper_init(64)
    c1 = O.widen_bf16(O.mult_nn_bf16(O.round_bf16(pa), pb.astype(np.complex64)))
    assert np.all(c1 == 1.0)
    b = latgen.random_b(seed=102)
    c16 = O.mult_nn_bf16(a16, O.round_f32(b))
    c = O.widen_bf16(c16)
    exact = O.mult_nn(O.widen_bf16(a16), O.round_f32(b).astype(np.complex128))
    ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(exact.view(np.float64)), 2 ** -126))) - 7)
    assert np.all(np.abs(c.view(np.float64) - exact.view(np.float64)) <= ulp)
    assert O.max_abs_diff(c, O.mult_nn(a, b)) <= 1e-2


def test_r12_form_emulator(O):
    """Reconstruct-12 emulator: with b = I rows 0-1 come back exactly, and on
    SU(3) inputs the result is within 1e-5 of the FP64 definition."""
    a = latgen.random_lattice(1024, seed=111)
    p = O.pack_r12(a)
    eye32 = latgen.identity_b().astype(np.complex64)
    c = O.mult_nn_r12(p, eye32)
    assert np.array_equal(c[:, :, :2, :], p)
    b = latgen.random_b(seed=112)
    c = O.mult_nn_r12(p, O.round_f32(b))
    assert O.max_abs_diff(c.astype(np.complex128), O.mult_nn(a, b)) <= 1e-5


# ----------------------------------------------------------------- SoA (O6)

def test_soa_transform_is_numpy_transpose(O):
    """P9: AoS -> SoA equals numpy's (1, 2, 3, 0) transpose, bit for bit, for
    both element sizes; the round trip is the identity."""
    a = latgen.random_lattice(777, seed=121)
    s = O.aos_to_soa(a)
    assert np.array_equal(s, np.ascontiguousarray(a.transpose(1, 2, 3, 0)))
    assert np.array_equal(O.soa_to_aos(s), a)
    a32 = a.astype(np.complex64)
    s32 = O.aos_to_soa(a32)
    assert np.array_equal(s32, np.ascontiguousarray(a32.transpose(1, 2, 3, 0)))
    assert np.array_equal(O.soa_to_aos(s32), a32)


# -------------------------------------------------------------- paper sizes

def test_paper_sizes_and_flop_count():
    """The byte and flop conventions used for reporting equal the paper's."""
    g = _golden("paper_sizes.txt")
    assert 9 * 2 * 4 == g["su3_matrix_bytes_f32"] and 9 * 2 * 8 == g["su3_matrix_bytes_f64"]
    assert 4 * g["su3_matrix_bytes_f32"] == g["b_bytes_f32"]
    assert 4 * g["su3_matrix_bytes_f64"] == g["b_bytes_f64"]
    # 4 links x 27 complex multiply-adds x (4 mul + 4 add)
    assert 4 * 27 * 8 == g["flop_per_site"]
    assert g["flop_per_site"] / (2 * g["site_bytes_f32"]) == pytest.approx(g["ai_f32"])
    assert g["flop_per_site"] / (2 * g["site_bytes_f64"]) == pytest.approx(g["ai_f64"])


def _hand_expanded(a, b):
    """Every entry written out: c_kl = a_k0 b_0l + a_k1 b_1l + a_k2 b_2l."""
    c = np.empty_like(a)
    for s in range(a.shape[0]):
        for j in range(4):
            A, B = a[s, j], b[j]
            c[s, j, 0, 0] = A[0, 0] * B[0, 0] + A[0, 1] * B[1, 0] + A[0, 2] * B[2, 0]
            c[s, j, 0, 1] = A[0, 0] * B[0, 1] + A[0, 1] * B[1, 1] + A[0, 2] * B[2, 1]
            c[s, j, 0, 2] = A[0, 0] * B[0, 2] + A[0, 1] * B[1, 2] + A[0, 2] * B[2, 2]
            c[s, j, 1, 0] = A[1, 0] * B[0, 0] + A[1, 1] * B[1, 0] + A[1, 2] * B[2, 0]
            c[s, j, 1, 1] = A[1, 0] * B[0, 1] + A[1, 1] * B[1, 1] + A[1, 2] * B[2, 1]
            c[s, j, 1, 2] = A[1, 0] * B[0, 2] + A[1, 1] * B[1, 2] + A[1, 2] * B[2, 2]
            c[s, j, 2, 0] = A[2, 0] * B[0, 0] + A[2, 1] * B[1, 0] + A[2, 2] * B[2, 0]
            c[s, j, 2, 1] = A[2, 0] * B[0, 1] + A[2, 1] * B[1, 1] + A[2, 2] * B[2, 1]
            c[s, j, 2, 2] = A[2, 0] * B[0, 2] + A[2, 1] * B[1, 2] + A[2, 2] * B[2, 2]
    return c


def test_hand_expanded_2_4_lattice(O):
    """The 3x3 products written out entry by entry on a 2^4 lattice (16 sites
    x 4 links) agree with the oracle to 1e-15."""
    a = latgen.random_lattice(2 ** 4, seed=131)
    b = latgen.random_b(seed=132)
    assert O.max_abs_diff(O.mult_nn(a, b), _hand_expanded(a, b)) <= 1e-15
