"""MI355X-native quaternion GEMM (placeholder; binding added with the C-ABI)."""


def flops(M, N, K):
    """Effective real flops of one M x N x K quaternion GEMM: 16 real
    multiply-adds per quaternion multiply-add (Tab. hc_flops), 2 flops each."""
    return 32 * int(M) * int(N) * int(K)
