"""Independent cross-check routes used by the oracle pins (CPU, numpy/torch).

None of these call the oracle or the GPU library; they rebuild results from
other statements in the paper: the basis multiplication table, the 2x2 complex
representation of a quaternion and of a quaternion matrix, and the complex
sub-algebra.  Storage convention: (cols, ld, 4) arrays, see ``workloads``.
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def basis_table():
    """T[i, j] = components of e_i e_j from tests/golden/basis_products.txt."""
    T = np.zeros((4, 4, 4))
    for line in open(os.path.join(GOLDEN, "basis_products.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        i, j = int(line[0]), int(line[1])
        T[i, j] = [float(x) for x in line[2:6]]
    return T


_T = None


def bf_mul(p, q):
    """p q by bilinear expansion over the basis table: sum_ij p_i q_j (e_i e_j)."""
    global _T
    if _T is None:
        _T = basis_table()
    out = [0.0, 0.0, 0.0, 0.0]
    for i in range(4):
        for j in range(4):
            for k in range(4):
                if _T[i, j, k] != 0.0:
                    out[k] += _T[i, j, k] * p[i] * q[j]
    return out


def bf_conj(q):
    return [q[0], -q[1], -q[2], -q[3]]


def logical(X, rows, cols):
    """(rows, cols, 4) logical view of a (cols, ld, 4) storage array."""
    return np.asarray(X)[:cols, :rows, :].transpose(1, 0, 2)


def apply_op(op, X, rows, cols):
    """Logical op(X) (rows x cols) from the stored operand (pure index/sign work)."""
    if op in ("N", "R"):
        L = logical(X, rows, cols).astype(np.float64)
    else:
        L = logical(X, cols, rows).astype(np.float64).transpose(1, 0, 2)
    if op in ("C", "R"):
        L = L * np.array([1.0, -1.0, -1.0, -1.0])
    return L


def bf_qgemm(opA, opB, M, N, K, alpha, A, B, beta, C):
    """Brute-force pure-Python quaternion GEMM for tiny sizes.  Returns logical
    (M, N, 4).  C is a logical (M, N, 4) array.  The sum is formed with the basis
    table product, then alpha and beta multiply from the left."""
    a = apply_op(opA, A, M, K)
    b = apply_op(opB, B, K, N)
    bz = all(x == 0.0 for x in beta)
    out = np.zeros((M, N, 4))
    for mu in range(M):
        for nu in range(N):
            acc = [0.0] * 4
            for ka in range(K):
                t = bf_mul(a[mu, ka], b[ka, nu])
                acc = [acc[c] + t[c] for c in range(4)]
            s = bf_mul(alpha, acc)
            u = [0.0] * 4 if bz else bf_mul(beta, C[mu, nu])
            out[mu, nu] = [s[c] + u[c] for c in range(4)]
    return out


def complex_rep_scalar(q):
    """2x2 complex representation of a quaternion (Sec. 2.1, Eq. h_matrep)."""
    z0 = q[0] + 1j * q[1]
    z1 = q[2] + 1j * q[3]
    return np.array([[z0, z1], [-np.conj(z1), np.conj(z0)]])


def complex_rep_pauli(q):
    """Same representation built from the Pauli basis map e0->s0, e1->i s3,
    e2->i s2, e3->i s1 (Sec. 2.1, Eq. pauli)."""
    s0 = np.eye(2, dtype=complex)
    s1 = np.array([[0, 1], [1, 0]], dtype=complex)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
    s3 = np.array([[1, 0], [0, -1]], dtype=complex)
    return q[0] * s0 + q[1] * 1j * s3 + q[2] * 1j * s2 + q[3] * 1j * s1


def complex_rep_block(Q):
    """Block form [[Q0_, Q1_], [-conj(Q1_), conj(Q0_)]] of a logical (R, S, 4)
    quaternion matrix, with Q0_ = Q^0 + i Q^1 and Q1_ = Q^2 + i Q^3
    (Sec. 2.2, Eq. qmat_complex, right-hand form)."""
    Q = np.asarray(Q, dtype=np.float64)
    Z0 = Q[..., 0] + 1j * Q[..., 1]
    Z1 = Q[..., 2] + 1j * Q[..., 3]
    return np.block([[Z0, Z1], [-np.conj(Z1), np.conj(Z0)]])


def complex_rep_kron(Q):
    """Kronecker form sum_i Q^i (x) (image of e_i) of Eq. qmat_complex."""
    Q = np.asarray(Q, dtype=np.float64)
    s0 = np.eye(2, dtype=complex)
    s1 = np.array([[0, 1], [1, 0]], dtype=complex)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
    s3 = np.array([[1, 0], [0, -1]], dtype=complex)
    return (np.kron(Q[..., 0], s0) + np.kron(Q[..., 1], 1j * s3)
            + np.kron(Q[..., 2], 1j * s2) + np.kron(Q[..., 3], 1j * s1))


def from_complex_block(Zc, R, S):
    """Inverse of complex_rep_block: read Q back from the top block row."""
    Z0 = Zc[:R, :S]
    Z1 = Zc[:R, S:]
    return np.stack([Z0.real, Z0.imag, Z1.real, Z1.imag], axis=-1)


def scalar_block(q, n):
    """Representation of the scalar matrix q*I_n in block form."""
    return complex_rep_block(np.broadcast_to(np.asarray(q, dtype=np.float64), (n, n, 4))
                             * np.eye(n)[:, :, None])


def qgemm_via_complex(opA, opB, M, N, K, alpha, A, B, beta, C):
    """alpha op(A) op(B) + beta C through complex128 matrix products on the
    block representation (Sec. 2.2, Eq. hc_mat_mult).  C is logical (M, N, 4)."""
    Ac = complex_rep_block(apply_op(opA, A, M, K))
    Bc = complex_rep_block(apply_op(opB, B, K, N))
    P = Ac @ Bc
    out = scalar_block(alpha, M) @ P
    if any(x != 0.0 for x in beta):
        out = out + scalar_block(beta, M) @ complex_rep_block(C)
    return from_complex_block(out, M, N)
