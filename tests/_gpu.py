"""Helpers for the GPU tests: device tensors from the seeded generator, NaN
poisoned outputs with guard regions, and case labels printed before each GPU
step."""

import functools
import sys

import numpy as np
import torch

GUARD = 64  # guard sites on each side of a poisoned output


def dev():
    return torch.device("cuda:0")


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def poisoned(shape, dtype):
    """An output tensor inside a larger NaN-filled buffer: returns (view,
    whole). The GUARD sites before and after the view must stay NaN."""
    whole = torch.empty((shape[0] + 2 * GUARD,) + tuple(shape[1:]), dtype=dtype, device=dev())
    if dtype == torch.bfloat16:
        whole.view(torch.int16).fill_(0x7FC1)       # a BF16 quiet NaN pattern
    elif dtype.is_complex:
        whole.view(torch.float64 if dtype == torch.complex128 else torch.float32).fill_(float("nan"))
    else:
        whole.fill_(float("nan"))
    return whole[GUARD:GUARD + shape[0]], whole


def poison_(t):
    """Fill t in place with NaN (BF16: the 0x7FC1 quiet-NaN pattern), so that
    any output element a kernel fails to write shows up."""
    if t.dtype == torch.bfloat16:
        t.view(torch.int16).fill_(0x7FC1)
    elif t.dtype.is_complex:
        torch.view_as_real(t).fill_(float("nan"))
    else:
        t.fill_(float("nan"))
    return t


def guards_intact(whole):
    g = torch.cat([whole[:GUARD].reshape(-1), whole[-GUARD:].reshape(-1)])
    if g.dtype == torch.bfloat16:
        return bool((g.view(torch.int16) == 0x7FC1).all())
    if g.is_complex():
        g = torch.view_as_real(g)
    return bool(torch.isnan(g).all())


def all_finite(t):
    if t.is_complex():
        t = torch.view_as_real(t)
    return bool(torch.isfinite(t.float() if t.dtype == torch.bfloat16 else t).all())


def bf16_bits(t):
    """BF16 tensor -> numpy uint16 bit patterns."""
    return t.contiguous().view(torch.int16).cpu().numpy().view(np.uint16)


L48 = 48 ** 4


@functools.lru_cache(maxsize=1)
def l48_case():
    """The benchmark's L=48 lattice (5,308,416 sites; a from seed 1, b from
    seed 2) and the oracle's FP64 product of the two, built once per session
    (3.06 GB each on the host)."""
    import latgen
    import oracle
    a = latgen.random_lattice(L48, seed=1)
    b = latgen.random_b(seed=2)
    return a, b, oracle.default().mult_nn(a, b)
