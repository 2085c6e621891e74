"""Seeded synthetic inputs for the SU(3) link multiply.

This module is the only code that both the GPU path's tests and the oracle's
tests consume. It draws random numbers and builds structured fixtures; it holds
none of the link multiply's arithmetic (no matrix products, no third-row
reconstruction).

Random source: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-based:

    key      = splitmix64(seed)
    word(n)  = splitmix64(key + n)               (mod 2**64)
    u(n)     = ((word(n) >> 11) + 0.5) * 2**-53  in the open interval (0, 1)

where splitmix64(x) adds the golden-ratio increment 0x9E3779B97F4A7C15 and then
applies the published 64-bit finaliser.  Gaussian entries come from the
Box-Muller transform of the uniform pair (u(2e), u(2e+1)).  Entry e of matrix m
is complex entry number 9*m + e (row-major 3x3), so the value of any entry is
a pure function of (seed, m, e): chunking and thread count never change it.

Lattice convention (paper, Background / SU3_Bench): sites = L**4, each site
holds four links (one per direction j = 0..3), each link a 3x3 complex matrix
stored row-major with interleaved (re, im).  Matrix m = 4*s + j for the a
lattice; m = j for the four constant b matrices.

Haar SU(3): a 3x3 complex Gaussian matrix is orthonormalised row by row
(Gram-Schmidt with <u, v> = sum conj(u) v, each projection applied twice as
in Giraud, Langou & Rozloznik 2005 so orthogonality holds to rounding), which
is the positive-diagonal QR construction and gives Haar-distributed U(3)
(Mezzadri, "How to generate random matrices from the classical compact
groups", Notices AMS 2007).  The third row
is then multiplied by conj(det U), which maps Haar U(3) onto Haar SU(3) (the map
commutes with left multiplication by SU(3)).  For a matrix of SU(3) that third
row equals the conjugate cross product of the first two; it is computed here
without that identity so that the reconstruct-12 tests have an independent
reference.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "uniform",
    "complex_gaussian",
    "haar_su3",
    "random_lattice",
    "random_b",
    "complex_normal_lattice",
    "identity_b",
    "permutation_b",
    "paper_init",
    "index_coded",
    "lattice_sites",
]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Default chunk of matrices per generation task and worker count.
_CHUNK = 1 << 19
_WORKERS = max(1, min(16, os.cpu_count() or 1))


def lattice_sites(L: int) -> int:
    """Number of sites of an L^4 lattice."""
    return int(L) ** 4


def _splitmix64_scalar(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = x + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, ctr: np.ndarray) -> np.ndarray:
    """u(n) in (0, 1) for each counter n (uint64 array)."""
    key = np.uint64(_splitmix64_scalar(int(seed) & _MASK64))
    with np.errstate(over="ignore"):
        w = _splitmix64(key + ctr.astype(np.uint64, copy=False))
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def complex_gaussian(seed: int, first_entry: int, count: int) -> np.ndarray:
    """`count` complex entries, each re/im standard normal N(0, 1).

    Entry n uses uniforms (2n, 2n+1) with the Box-Muller transform.
    """
    n = np.arange(first_entry, first_entry + count, dtype=np.uint64)
    u1 = uniform(seed, n * np.uint64(2))
    u2 = uniform(seed, n * np.uint64(2) + np.uint64(1))
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    out = np.empty(count, dtype=np.complex128)
    out.real = r * np.cos(t)
    out.imag = r * np.sin(t)
    return out


def _det3(u: np.ndarray) -> np.ndarray:
    """Determinant of a stack of 3x3 complex matrices (cofactor expansion)."""
    return (u[:, 0, 0] * (u[:, 1, 1] * u[:, 2, 2] - u[:, 1, 2] * u[:, 2, 1])
            - u[:, 0, 1] * (u[:, 1, 0] * u[:, 2, 2] - u[:, 1, 2] * u[:, 2, 0])
            + u[:, 0, 2] * (u[:, 1, 0] * u[:, 2, 1] - u[:, 1, 1] * u[:, 2, 0]))


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / np.sqrt(np.sum(v.real ** 2 + v.imag ** 2, axis=1, keepdims=True))


def _proj(r: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Component of each row v along the unit row r: <r, v> r."""
    return np.sum(np.conj(r) * v, axis=1, keepdims=True) * r


def _haar_chunk(seed: int, m0: int, count: int) -> np.ndarray:
    g = complex_gaussian(seed, 9 * m0, 9 * count).reshape(count, 3, 3)
    r0 = _normalise(g[:, 0, :])
    v1 = g[:, 1, :]
    for _ in range(2):  # project twice: keeps rows orthogonal to ~1 ulp
        v1 = v1 - _proj(r0, v1)
    r1 = _normalise(v1)
    v2 = g[:, 2, :]
    for _ in range(2):
        v2 = v2 - _proj(r0, v2)
        v2 = v2 - _proj(r1, v2)
    r2 = _normalise(v2)
    u = np.stack([r0, r1, r2], axis=1)
    d = _det3(u)
    d = d / np.abs(d)  # unit phase; guards against a rounding drift in |det|
    u[:, 2, :] *= np.conj(d)[:, None]
    return u


def haar_su3(seed: int, first_matrix: int, count: int, out: np.ndarray | None = None) -> np.ndarray:
    """Haar-random SU(3) matrices number first_matrix .. first_matrix+count-1.

    Returns a (count, 3, 3) complex128 array (written into `out` if given).
    Generation is split into chunks run on a thread pool; values do not depend
    on the split.
    """
    if out is None:
        out = np.empty((count, 3, 3), dtype=np.complex128)
    if count == 0:
        return out
    starts = list(range(0, count, _CHUNK))

    def work(off: int) -> None:
        n = min(_CHUNK, count - off)
        out[off:off + n] = _haar_chunk(seed, first_matrix + off, n)

    if len(starts) == 1:
        work(0)
    else:
        with ThreadPoolExecutor(max_workers=_WORKERS) as ex:
            list(ex.map(work, starts))
    return out


def random_lattice(sites: int, seed: int = 1) -> np.ndarray:
    """a[s][j] Haar SU(3), as a (sites, 4, 3, 3) complex128 array (site-major)."""
    a = np.empty((sites, 4, 3, 3), dtype=np.complex128)
    haar_su3(seed, 0, 4 * sites, out=a.reshape(4 * sites, 3, 3))
    return a


def random_b(seed: int = 2) -> np.ndarray:
    """b[j], j = 0..3: four Haar SU(3) matrices, (4, 3, 3) complex128."""
    return haar_su3(seed, 0, 4)


def complex_normal_lattice(sites: int, seed: int = 3) -> np.ndarray:
    """(sites, 4, 3, 3) circular standard complex normal entries, E|z|^2 = 1.

    Used for the upstream gradient dC: re and im are each N(0, 1/2).
    """
    n = sites * 36
    out = np.empty(n, dtype=np.complex128)
    starts = list(range(0, n, 9 * _CHUNK))
    scale = np.sqrt(0.5)

    def work(off: int) -> None:
        k = min(9 * _CHUNK, n - off)
        out[off:off + k] = complex_gaussian(seed, off, k) * scale

    if len(starts) == 1:
        work(0)
    else:
        with ThreadPoolExecutor(max_workers=_WORKERS) as ex:
            list(ex.map(work, starts))
    return out.reshape(sites, 4, 3, 3)


def identity_b() -> np.ndarray:
    """b[j] = I for every j."""
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (4, 3, 3)).copy()


def permutation_b() -> np.ndarray:
    """Four distinct SU(3) matrices with entries in {0, +-1, +-i}.

    b[0] = I, b[1] = P (cyclic shift, det +1), b[2] = P^2 written out,
    b[3] = diag(i, i, -1) (det = i*i*(-1) = 1).  Each is neither symmetric
    in the b vs b^T sense (except b[0] and b[3]) nor equal to another, so a
    transposed b or a wrong link index changes the product; every product
    entry is an exact copy of an a entry up to a sign or a factor i.
    """
    b = np.zeros((4, 3, 3), dtype=np.complex128)
    b[0] = np.eye(3)
    # P maps column l of the product to column l-1 of a: P[m, l] = 1 if m == (l+1) % 3
    for l in range(3):
        b[1, (l + 1) % 3, l] = 1.0
        b[2, (l + 2) % 3, l] = 1.0
    b[3] = np.diag([1j, 1j, -1.0])
    return b


def paper_init(sites: int) -> tuple[np.ndarray, np.ndarray]:
    """The paper's benchmark initialisation (Performance on Xeon, the
    initialisation calls listed with the per-socket memory table): every entry
    of every a link is 1+0i and every entry of every b link is 1/3+0i."""
    a = np.full((sites, 4, 3, 3), 1.0 + 0.0j, dtype=np.complex128)
    b = np.full((4, 3, 3), 1.0 / 3.0 + 0.0j, dtype=np.complex128)
    return a, b


def index_coded(sites: int) -> np.ndarray:
    """a[s][j][k][l] = q + i*(-q - 0.5) with q = ((s*4+j)*3+k)*3+l, reduced
    modulo 2**22 so the values stay exact in FP32 (and in FP64)."""
    q = (np.arange(sites * 36, dtype=np.int64) % (1 << 22)).astype(np.float64)
    out = np.empty(sites * 36, dtype=np.complex128)
    out.real = q
    out.imag = -q - 0.5
    return out.reshape(sites, 4, 3, 3)
