"""MI355X (gfx950) SU(3) link multiply: HIP kernels behind a C ABI
(include/su3.h, libsu3.so) with a thin PyTorch front end.

    from paper_2103_00571_amd import ops
    c = ops.mult_nn(a, b)          # c[s][j] = a[s][j] @ b[j]

The package fails on import when libsu3.so is missing; there is no other
implementation to fall back to.
"""

from . import abi, ops  # noqa: F401
from .ops import (SU3_BF16, SU3_F32, SU3_F64, SU3_R12_F32, SU3MultNN, aos_to_soa,  # noqa: F401
                  mult_nn, mult_nn_autograd, mult_nn_bwd, mult_nn_soa, pack, soa_to_aos, unpack)

__version__ = "0.1.0"
