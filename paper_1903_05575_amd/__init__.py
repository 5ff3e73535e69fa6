"""MI355X-native quaternion GEMM: C <- alpha op(A) op(B) + beta C.

The computation runs in hand-written HIP kernels for gfx950 behind the C ABI
of ``libqgemm.so`` (include/qgemm.h).  This package is the thin Python
binding: it marshals torch GPU tensors (used only for device memory and
streams) to that ABI.

Storage: a rows x cols quaternion matrix with leading dimension ld is a
contiguous tensor of shape (cols, ld, 4): column-major, four interleaved
components (q0, q1, q2, q3) per element.
"""
from ._lib import (QGemmError, GroupedPlan, TILE_CLASSES, lib, qgemm_d, qgemm_s, qgemm_ex,  # noqa: F401
                   qherk, qtrmm, qgemm_mixed, qaxpy, qdot, qgemv, qgemm_backward,
                   exported_symbols)
from .autograd import QGemmFn, QLinear, qgemm  # noqa: F401


def flops(M, N, K):
    """Effective real flops of one M x N x K quaternion GEMM: 16 real
    multiply-adds per quaternion multiply-add (Tab. hc_flops), 2 flops each."""
    return 32 * int(M) * int(N) * int(K)
