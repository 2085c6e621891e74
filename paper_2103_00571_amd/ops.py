"""Torch-facing front end of libsu3: shape and dtype checks, output
allocation with torch.empty, and the current HIP stream. PyTorch supplies
device memory and streams only; every computation is a libsu3 kernel.

Tensor forms (site-major "AoS", one row per site, see include/su3.h):

    form          a                              b                  c
    SU3_F64       complex128 (N, 4, 3, 3)        complex128 (4,3,3)  like a
    SU3_F32       complex64  (N, 4, 3, 3)        complex64 (4,3,3)   like a
    SU3_BF16      bfloat16   (N, 4, 3, 3, 2)     complex64 (4,3,3)   like a
    SU3_R12_F32   complex64  (N, 4, 2, 3)        complex64 (4,3,3)   complex64 (N,4,3,3)
    SU3_R12C_F32  complex64  (N, 4, 2, 3)        complex64 (4,3,3)   complex64 (N,4,2,3)
    SU3_R12_F64   complex128 (N, 4, 2, 3)        complex128 (4,3,3)  complex128 (N,4,3,3)

SU3_R12C_F32 stores a exactly like SU3_R12_F32; pass form=SU3_R12C_F32 to
keep the product compressed. SoA tensors are (4, 3, 3, P) in complex128 or
complex64, P = N for the dense layout or a padded pitch P > N (soa_pitch).
"""

from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import abi
from .abi import SU3_BF16, SU3_F32, SU3_F64, SU3_R12_F32, SU3_R12_F64, SU3_R12C_F32, check

__all__ = [
    "SU3_F64", "SU3_F32", "SU3_BF16", "SU3_R12_F32", "SU3_R12C_F32", "SU3_R12_F64",
    "form_of", "mult_nn", "mult_na", "mult_an", "mat_vec", "mult_nn_soa", "soa_pitch", "aos_to_soa", "soa_to_aos",
    "pack", "unpack",
    "mult_nn_bwd", "mult_nn_bwd_workspace", "stream_copy", "stream_shape", "SU3MultNN", "mult_nn_autograd",
    "launch_shape",
]

_B_DTYPE = {SU3_F64: torch.complex128, SU3_F32: torch.complex64, SU3_BF16: torch.complex64,
            SU3_R12_F32: torch.complex64, SU3_R12C_F32: torch.complex64, SU3_R12_F64: torch.complex128}


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _need_gpu(*ts: torch.Tensor) -> None:
    dev = ts[0].device
    for t in ts:
        if t.device.type != "cuda":
            raise ValueError("libsu3 works on GPU tensors; got a tensor on %s" % t.device)
        if t.device != dev:
            raise ValueError("all tensors must be on one device")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if t.is_conj() or t.is_neg():
            # a lazy conjugate or negative view shares the memory of its base,
            # which holds the unconjugated values
            raise ValueError("tensors must not be lazy conjugate or negative views; call .resolve_conj() "
                             "and .resolve_neg() first")


def form_of(a: torch.Tensor) -> int:
    """Storage form of an AoS lattice tensor, from its dtype and shape."""
    if a.dtype == torch.complex128 and a.dim() == 4 and tuple(a.shape[1:]) == (4, 3, 3):
        return SU3_F64
    if a.dtype == torch.complex64 and a.dim() == 4 and tuple(a.shape[1:]) == (4, 3, 3):
        return SU3_F32
    if a.dtype == torch.bfloat16 and a.dim() == 5 and tuple(a.shape[1:]) == (4, 3, 3, 2):
        return SU3_BF16
    if a.dtype == torch.complex64 and a.dim() == 4 and tuple(a.shape[1:]) == (4, 2, 3):
        return SU3_R12_F32
    if a.dtype == torch.complex128 and a.dim() == 4 and tuple(a.shape[1:]) == (4, 2, 3):
        return SU3_R12_F64
    raise ValueError("not a lattice tensor: dtype %s shape %s" % (a.dtype, tuple(a.shape)))


def _c_shape(form: int, sites: int) -> tuple:
    if form == SU3_BF16:
        return (sites, 4, 3, 3, 2)
    if form == SU3_R12C_F32:
        return (sites, 4, 2, 3)
    return (sites, 4, 3, 3)


def _c_dtype(form: int) -> torch.dtype:
    return {SU3_F64: torch.complex128, SU3_F32: torch.complex64, SU3_BF16: torch.bfloat16,
            SU3_R12_F32: torch.complex64, SU3_R12C_F32: torch.complex64, SU3_R12_F64: torch.complex128}[form]


def _check_b(b: torch.Tensor, form: int) -> None:
    if b.dtype != _B_DTYPE[form] or tuple(b.shape) != (4, 3, 3):
        raise ValueError("b must be %s of shape (4, 3, 3) for this form" % _B_DTYPE[form])


def mult_nn(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
            form: int | None = None) -> torch.Tensor:
    """c[s][j] = a[s][j] @ b[j] on the site-major layout (any form; the form
    is taken from a unless given, which selects SU3_R12C_F32)."""
    inferred = form_of(a)
    if form is None:
        form = inferred
    elif not (form == inferred or (form == SU3_R12C_F32 and inferred == SU3_R12_F32)):
        raise ValueError("a is not stored in form %d" % form)
    _check_b(b, form)
    sites = a.shape[0]
    if out is None:
        out = torch.empty(_c_shape(form, sites), dtype=_c_dtype(form), device=a.device)
    elif out.dtype != _c_dtype(form) or tuple(out.shape) != _c_shape(form, sites):
        raise ValueError("out has the wrong dtype or shape")
    _need_gpu(a, b, out)
    with torch.cuda.device(a.device):
        check(abi.su3_mult_nn(a.data_ptr(), b.data_ptr(), out.data_ptr(), sites, form, _stream(a)),
              "su3_mult_nn")
    return out


def _mult_other(fn, name: str, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None) -> torch.Tensor:
    form = form_of(a)
    if form not in (SU3_F64, SU3_F32):
        raise ValueError("%s exists for FP64 and FP32 links" % name)
    _check_b(b, form)
    if out is None:
        out = torch.empty_like(a)
    elif out.dtype != a.dtype or out.shape != a.shape:
        raise ValueError("out has the wrong dtype or shape")
    _need_gpu(a, b, out)
    with torch.cuda.device(a.device):
        check(fn(a.data_ptr(), b.data_ptr(), out.data_ptr(), a.shape[0], form, _stream(a)), name)
    return out


def mult_na(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """c[s][j] = a[s][j] @ b[j]^H (FP64, FP32)."""
    return _mult_other(abi.su3_mult_na, "su3_mult_na", a, b, out)


def mult_an(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """c[s][j] = a[s][j]^H @ b[j] (FP64, FP32)."""
    return _mult_other(abi.su3_mult_an, "su3_mult_an", a, b, out)


def mat_vec(a: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """w[s][j] = a[s][j] @ v[s]: a (N, 4, 3, 3), v (N, 3), w (N, 4, 3), FP64 or FP32."""
    form = form_of(a)
    if form not in (SU3_F64, SU3_F32):
        raise ValueError("mat_vec exists for FP64 and FP32 links")
    sites = a.shape[0]
    if v.dtype != a.dtype or tuple(v.shape) != (sites, 3):
        raise ValueError("v must be (sites, 3) of a's dtype")
    if out is None:
        out = torch.empty((sites, 4, 3), dtype=a.dtype, device=a.device)
    elif out.dtype != a.dtype or tuple(out.shape) != (sites, 4, 3):
        raise ValueError("out has the wrong dtype or shape")
    _need_gpu(a, v, out)
    with torch.cuda.device(a.device):
        check(abi.su3_mat_vec(a.data_ptr(), v.data_ptr(), out.data_ptr(), sites, form, _stream(a)), "su3_mat_vec")
    return out


def _soa_form(x: torch.Tensor) -> int:
    if x.dim() == 4 and tuple(x.shape[:3]) == (4, 3, 3):
        if x.dtype == torch.complex128:
            return SU3_F64
        if x.dtype == torch.complex64:
            return SU3_F32
    raise ValueError("not an SoA lattice tensor: dtype %s shape %s" % (x.dtype, tuple(x.shape)))


def soa_pitch(sites: int, form: int) -> int:
    """Plane pitch of the padded SoA layout at which mult_nn_soa streams at the
    site-major rate (su3_soa_pitch)."""
    return abi.su3_soa_pitch(sites, form)


def mult_nn_soa(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
                sites: int | None = None) -> torch.Tensor:
    """The same product on the SoA layout, (4, 3, 3, P) planes. The first
    `sites` elements of each plane are the lattice (default: all P); with
    sites < P the layout is padded and the padding is neither read nor
    written."""
    form = _soa_form(a)
    _check_b(b, form)
    pitch = a.shape[3]
    sites = pitch if sites is None else sites
    if not 0 <= sites <= pitch:
        raise ValueError("sites must lie in [0, pitch]")
    if out is None:
        out = torch.empty_like(a)
    elif out.dtype != a.dtype or out.shape != a.shape:
        raise ValueError("out has the wrong dtype or shape")
    _need_gpu(a, b, out)
    with torch.cuda.device(a.device):
        if sites == pitch:
            rc = abi.su3_mult_nn_soa(a.data_ptr(), b.data_ptr(), out.data_ptr(), sites, form, _stream(a))
        else:
            rc = abi.su3_mult_nn_soa_pitched(a.data_ptr(), b.data_ptr(), out.data_ptr(), sites, pitch, form,
                                             _stream(a))
        check(rc, "su3_mult_nn_soa")
    return out


def aos_to_soa(x: torch.Tensor, pitch: int | None = None) -> torch.Tensor:
    """Site-major links -> SoA planes (4, 3, 3, pitch); pitch defaults to the
    site count (the dense layout). Padding elements are left uninitialised."""
    form = form_of(x)
    if form not in (SU3_F64, SU3_F32):
        raise ValueError("SoA exists for FP64 and FP32 only")
    sites = x.shape[0]
    pitch = sites if pitch is None else pitch
    if pitch < sites:
        raise ValueError("pitch must be at least the site count")
    out = torch.empty((4, 3, 3, pitch), dtype=x.dtype, device=x.device)
    _need_gpu(x, out)
    with torch.cuda.device(x.device):
        check(abi.su3_aos_to_soa_pitched(x.data_ptr(), out.data_ptr(), sites, pitch, form, _stream(x)),
              "su3_aos_to_soa")
    return out


def soa_to_aos(x: torch.Tensor, sites: int | None = None) -> torch.Tensor:
    """SoA planes (4, 3, 3, P) -> site-major links of the first `sites`
    elements of each plane (default: all P)."""
    form = _soa_form(x)
    pitch = x.shape[3]
    sites = pitch if sites is None else sites
    if not 0 <= sites <= pitch:
        raise ValueError("sites must lie in [0, pitch]")
    out = torch.empty((sites, 4, 3, 3), dtype=x.dtype, device=x.device)
    _need_gpu(x, out)
    with torch.cuda.device(x.device):
        check(abi.su3_soa_to_aos_pitched(x.data_ptr(), out.data_ptr(), sites, pitch, form, _stream(x)),
              "su3_soa_to_aos")
    return out


def _packed_spec(form: int, sites: int) -> tuple[tuple, torch.dtype]:
    if form == SU3_F64:
        return (sites, 4, 3, 3), torch.complex128
    if form == SU3_F32:
        return (sites, 4, 3, 3), torch.complex64
    if form == SU3_BF16:
        return (sites, 4, 3, 3, 2), torch.bfloat16
    if form in (SU3_R12_F32, SU3_R12C_F32):
        return (sites, 4, 2, 3), torch.complex64
    if form == SU3_R12_F64:
        return (sites, 4, 2, 3), torch.complex128
    raise ValueError("unknown form %r" % form)


def pack(a64: torch.Tensor, form: int) -> torch.Tensor:
    """FP64 AoS links -> storage form `form` (rounding to nearest even)."""
    if form_of(a64) != SU3_F64:
        raise ValueError("pack takes FP64 (complex128) links")
    shape, dtype = _packed_spec(form, a64.shape[0])
    out = torch.empty(shape, dtype=dtype, device=a64.device)
    _need_gpu(a64, out)
    with torch.cuda.device(a64.device):
        check(abi.su3_pack(a64.data_ptr(), out.data_ptr(), a64.shape[0], form, _stream(a64)), "su3_pack")
    return out


def unpack(x: torch.Tensor, form: int | None = None) -> torch.Tensor:
    """Storage form -> FP64 AoS links (R12 rebuilds row 2 in FP64)."""
    inferred = form_of(x)
    form = inferred if form is None else form
    if not (form == inferred or (form == SU3_R12C_F32 and inferred == SU3_R12_F32)):
        raise ValueError("tensor is not in form %d" % form)
    out = torch.empty((x.shape[0], 4, 3, 3), dtype=torch.complex128, device=x.device)
    _need_gpu(x, out)
    with torch.cuda.device(x.device):
        check(abi.su3_unpack(x.data_ptr(), out.data_ptr(), x.shape[0], form, _stream(x)), "su3_unpack")
    return out


def mult_nn_bwd_workspace(sites: int, form: int, device: torch.device | int | None = None) -> torch.Tensor:
    """A workspace tensor large enough for mult_nn_bwd on `sites` sites."""
    nbytes = abi.su3_mult_nn_bwd_workspace_bytes(sites, form)
    return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=device)


def mult_nn_bwd(a: torch.Tensor, b: torch.Tensor, dc: torch.Tensor, da: torch.Tensor | None = None,
                db: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """Adjoint: returns (da, db64) with da = dc b^H per site (dtype of a) and
    db64 = sum_s a^H dc as complex128 (4, 3, 3), deterministic. da, db and the
    workspace ws (uint8, at least su3_mult_nn_bwd_workspace_bytes) may be
    passed in; whatever is missing is allocated with torch.empty."""
    form = form_of(a)
    if form not in (SU3_F64, SU3_F32):
        raise ValueError("the adjoint exists for FP64 and FP32")
    _check_b(b, form)
    if dc.dtype != a.dtype or dc.shape != a.shape:
        raise ValueError("dc must match a in dtype and shape")
    sites = a.shape[0]
    if da is None:
        da = torch.empty_like(a)
    elif da.dtype != a.dtype or da.shape != a.shape:
        raise ValueError("da must match a in dtype and shape")
    if db is None:
        db = torch.empty((4, 3, 3), dtype=torch.complex128, device=a.device)
    elif db.dtype != torch.complex128 or tuple(db.shape) != (4, 3, 3):
        raise ValueError("db must be complex128 of shape (4, 3, 3)")
    if ws is None:
        ws = mult_nn_bwd_workspace(sites, form, a.device)
    elif ws.dtype != torch.uint8 or ws.dim() != 1:
        raise ValueError("ws must be a 1-D uint8 tensor")
    _need_gpu(a, b, dc, da, db, ws)
    with torch.cuda.device(a.device):
        check(abi.su3_mult_nn_bwd(a.data_ptr(), b.data_ptr(), dc.data_ptr(), da.data_ptr(), db.data_ptr(), sites,
                                  form, ws.data_ptr(), ws.numel(), _stream(a)), "su3_mult_nn_bwd")
    return da, db


def stream_shape(a: torch.Tensor, b: torch.Tensor | None, c: torch.Tensor, in_a: int, in_b: int, out: int,
                 waves_per_cu: int = 0, tile_order: int = 0) -> None:
    """The streaming probe of an access shape (su3_stream_shape) over byte
    buffers: a holds tiles*1024*in_a bytes, b tiles*1024*in_b, c tiles*1024*out.
    tile_order 0 gives workgroup i tile i, 1 the XCD-contiguous order of the
    site-major products."""
    tiles = a.numel() * a.element_size() // (1024 * in_a)
    if (a.numel() * a.element_size() != tiles * 1024 * in_a or c.numel() * c.element_size() != tiles * 1024 * out
            or (in_b and (b is None or b.numel() * b.element_size() != tiles * 1024 * in_b))):
        raise ValueError("buffer sizes do not match the shape")
    ts = (a, c) if not in_b else (a, b, c)
    _need_gpu(*ts)
    with torch.cuda.device(a.device):
        check(abi.su3_stream_shape(a.data_ptr(), b.data_ptr() if in_b else None, c.data_ptr(), tiles, in_a, in_b,
                                   out, waves_per_cu, tile_order, _stream(a)), "su3_stream_shape")


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """dst <- src bytewise with the library's streaming copy kernel."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("size mismatch")
    _need_gpu(src, dst)
    with torch.cuda.device(src.device):
        check(abi.su3_stream_copy(src.data_ptr(), dst.data_ptr(), n, _stream(src)), "su3_stream_copy")
    return dst


def launch_shape(sites: int, form: int, device: torch.device | int | None = None) -> tuple[int, int]:
    """(workgroups, threads per workgroup) su3_mult_nn launches for this size."""
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        return abi.su3_launch_shape(sites, form)


class SU3MultNN(torch.autograd.Function):
    """c = a @ b[j] per site and link, differentiable in a and b (FP64, FP32).

    backward uses the library's fused adjoint: da = dc b^H and a deterministic
    FP64 site sum for db, returned in b's dtype."""

    @staticmethod
    def forward(ctx, a, b):
        ctx.save_for_backward(a, b)
        return mult_nn(a, b)

    @staticmethod
    @once_differentiable
    def backward(ctx, dc):
        a, b = ctx.saved_tensors
        # autograd may hand over a lazy conjugate view (after a .conj() in
        # the graph); the kernels need the values themselves
        da, db = mult_nn_bwd(a, b, dc.resolve_conj().resolve_neg().contiguous())
        return (da if ctx.needs_input_grad[0] else None,
                db.to(b.dtype) if ctx.needs_input_grad[1] else None)


def mult_nn_autograd(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return SU3MultNN.apply(a, b)
