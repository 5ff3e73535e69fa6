"""Helpers shared by the GPU parity tests: marshalling, error measures and the
componentwise rounding bounds each parity test asserts beside the relative
Frobenius bar.

Bounds.  For an output quaternion (mu, nu) let S = sum_k |op(A)_{mu k}|_1
|op(B)_{k nu}|_1 (|q|_1 = sum of the absolute components).  Every real of the
product, sum_k L(op(A)_{mu k}) op(B)_{k nu}, is a sum of 4K real products
whose absolute values add up to at most S, so S bounds what rounding can act
on.  With gamma(d) = d u / (1 - d u) (d roundings of relative size u):

  FP64 path:   (4K + 8) u64 (|alpha|_1 S + |beta|_1 |C|_1)

  split path (FP32 operands as three BF16 pieces h + m + l, epsilon = 2^-8):
    |h| <= (1 + e)|x|, |m| <= e (1 + e)|x|, |l| <= e^2 (1 + e)|x| and h + m + l
    = x exactly, so the piece products left out of a real product x y are at
    most drop(T) |x| |y|:
      T = 9: 0;  T = 6 (ml, lm, ll): (1 + e)^2 (2 e^3 + e^4);
      T = 3 (hl, mm, lh, ml, lm, ll): (1 + e)^2 (3 e^2 + 2 e^3 + e^4).
    Each piece product is exact in FP32 (8 x 8 significant bits) and the
    formed ones add up to at most rho2 |x| |y|, rho2 = ((1 + e)(1 + e + e^2))^2.
    They are summed in FP32: one accumulator takes the T products of every
    real product of a K-panel of 64 quaternions (256 T summands, fewer when K
    is smaller), then is added into a second accumulator once per panel.
    Whatever the order inside the matrix cores, a summand passes through at
    most d = min(4K, 256) T + ceil(K / 64) additions; each is taken to err by
    up to one FP32 ulp (u = 2^-23, any rounding mode).  The FP32 epilogue
    (alpha converted, 4-term Hamilton product, beta term, final add) adds at
    most 6 more roundings per path.  So
      |alpha|_1 S (drop(T) + rho2 gamma(d + 6)) + |beta|_1 |C|_1 gamma(6),
    with FP64 epilogue roundings (u64) for the FP64-output variant.
  Operations that scale an operand in FP32 before the split (a middle scalar,
  the conj(alpha) G operand of the gradient) add `pre` roundings to d.

A test asserts three things: the global relative Frobenius error under the
path's bar, every real within its componentwise bound, and the relative
Frobenius error of every block of 32 x 32 outputs under the same bar (so an
error confined to a few tiles cannot hide in the global norm).
"""
import math

import numpy as np
import torch

U64 = 2.0 ** -53
U32 = 2.0 ** -24
U_ACC32 = 2.0 ** -23
EPS_BF16 = 2.0 ** -8
SPLIT_PANEL = 64
SPLIT_BAR = {3: 3e-5, 6: 1e-6, 9: 1e-6}
F64_BAR = 1e-13


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def logical(X, rows, cols):
    return np.asarray(X)[:cols, :rows, :].transpose(1, 0, 2)


def relfro(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want)
    return np.linalg.norm(got - want) / (den if den > 0 else 1.0)


def norm1(X):
    """Per-element 1-norm of a logical (r, c, 4) quaternion matrix."""
    return np.abs(np.asarray(X, dtype=np.float64)).sum(-1)


def op_logical(op, X, rows, cols):
    """Logical op(X) (rows x cols) from a stored operand; magnitudes only
    matter here, so conjugation is not applied."""
    if op in ("N", "R"):
        return logical(X, rows, cols)
    return logical(X, cols, rows).transpose(1, 0, 2)


def qnorm1(q):
    return float(np.abs(np.asarray(q, dtype=np.float64)).sum())


def gamma(d, u):
    return d * u / (1.0 - d * u)


def mag_sum(a1, b1):
    """S = sum_k a1[mu, k] b1[k, nu] from per-element 1-norms (M x K, K x N)."""
    a1 = np.asarray(a1, dtype=np.float64)
    b1 = np.asarray(b1, dtype=np.float64)
    if a1.shape[1] == 0:
        return np.zeros((a1.shape[0], b1.shape[1]))
    return a1 @ b1


def split_drop(terms):
    e = EPS_BF16
    r = (1 + e) ** 2
    return {9: 0.0, 6: r * (2 * e ** 3 + e ** 4), 3: r * (3 * e ** 2 + 2 * e ** 3 + e ** 4)}[terms]


def split_depth(K, terms, panel=SPLIT_PANEL):
    return min(4 * K, 4 * panel) * terms + math.ceil(K / panel)


def bound_f64(S, K, alpha1, beta1=0.0, c1=0.0, extra=8):
    """(4K + extra) u64 (|alpha|_1 S + |beta|_1 |C|_1)."""
    cterm = beta1 * np.nan_to_num(c1) if beta1 != 0 else 0.0
    return (4 * K + extra) * U64 * (alpha1 * np.asarray(S) + cterm)


def bound_split(S, K, terms, alpha1, beta1=0.0, c1=0.0, pre=0, post=6, c64=False):
    """Componentwise bound of the split-BF16 path (module docstring)."""
    e = EPS_BF16
    rho2 = ((1 + e) * (1 + e + e * e)) ** 2
    d = split_depth(K, terms) + pre
    u_ep = U64 if c64 else U_ACC32
    coef = split_drop(terms) + rho2 * gamma(d, U_ACC32) + rho2 * gamma(post, u_ep)
    cterm = beta1 * np.nan_to_num(c1) * gamma(post, u_ep) if beta1 != 0 else 0.0
    return alpha1 * coef * np.asarray(S) + cterm


def gemm_S(p):
    """S of a GEMM problem dict (W.gemm_problem layout)."""
    M, N, K = p["M"], p["N"], p["K"]
    a1 = norm1(op_logical(p["opA"], p["A"], M, K)) if K else np.zeros((M, 0))
    b1 = norm1(op_logical(p["opB"], p["B"], K, N)) if K else np.zeros((0, N))
    return mag_sum(a1, b1)


def error_bound(p, u=U64, extra=8):
    """FP64 componentwise bound of a GEMM problem dict."""
    M, N = p["M"], p["N"]
    return bound_f64(gemm_S(p), p["K"], qnorm1(p["alpha"]), qnorm1(p["beta"]),
                     norm1(logical(p["C"], M, N)), extra)


def split_error_bound(p, terms=6, c64=False):
    """Split-path componentwise bound of a GEMM problem dict."""
    M, N = p["M"], p["N"]
    return bound_split(gemm_S(p), p["K"], terms, qnorm1(p["alpha"]), qnorm1(p["beta"]),
                       norm1(logical(p["C"], M, N)), c64=c64)


def worst_block_relfro(got, want, mask=None, block=32, min_count=64):
    """Largest relative Frobenius error over the block x block tiles of a
    logical (M, N, 4) result, counting only masked elements; tiles with fewer
    than min_count masked elements (or a zero reference) are skipped."""
    g = np.asarray(got, dtype=np.float64)
    w = np.asarray(want, dtype=np.float64)
    M, N = g.shape[:2]
    worst = 0.0
    for i in range(0, M, block):
        for j in range(0, N, block):
            gb, wb = g[i:i + block, j:j + block], w[i:i + block, j:j + block]
            if mask is not None:
                mb = mask[i:i + block, j:j + block]
                gb, wb = gb[mb], wb[mb]
            if gb.size < 4 * min_count:
                continue
            den = np.linalg.norm(wb)
            if den > 0:
                worst = max(worst, np.linalg.norm(gb - wb) / den)
    return worst


def assert_parity(got, want, bound, bar, mask=None, block=32, label="", verbose=True):
    """got, want: logical (M, N, 4); bound: (M, N) componentwise bound of each
    quaternion's four reals; bar: relative Frobenius bar.  With a mask only
    the selected elements are checked.  Returns (global error, largest ratio
    of an error to its componentwise bound, worst block error)."""
    g = np.asarray(got, dtype=np.float64)
    w = np.asarray(want, dtype=np.float64)
    b = np.broadcast_to(np.asarray(bound, dtype=np.float64), g.shape[:2])
    if mask is not None:
        gs, ws, bs = g[mask], w[mask], b[mask]
    else:
        gs, ws, bs = g.reshape(-1, 4), w.reshape(-1, 4), b.reshape(-1)
    assert np.isfinite(gs).all(), f"{label}: non-finite result"
    err = relfro(gs, ws)
    diff = np.abs(gs - ws)
    ratio = float((diff / (bs[:, None] + 1e-300)).max()) if diff.size else 0.0
    wb = worst_block_relfro(g, w, mask, block)
    if verbose:
        print(f"{label}: rel err {err:.3e}, worst {block}x{block} block {wb:.3e}, "
              f"max |err| / componentwise bound {ratio:.3e}")
    assert err <= bar, f"{label}: rel err {err:.3e} > {bar:.1e}"
    assert (diff <= bs[:, None] + 1e-300).all(), f"{label}: componentwise bound exceeded ({ratio:.3e}x)"
    assert wb <= bar, f"{label}: block rel err {wb:.3e} > {bar:.1e}"
    return err, ratio, wb


def split_pipeline(M, N):
    """The split launcher's pipeline for a full M x N output on device 0 (a
    mirror of its rule): TL3 (32 x 64 tiles, two LDS stages) when the 32-row
    grid fills the block slots (two per CU) more than 1.1x better than the
    64-row grid, else TL1 (64 x 64, one LDS stage, 16-quaternion K-tiles) for
    grids of fewer 64 x 64 tiles than slots, else TL2 (64 x 64, two stages,
    8-quaternion K-tiles)."""
    slots = 2 * torch.cuda.get_device_properties(0).multi_processor_count

    def fill(t):
        rounds = -(-t // slots)
        return t / (rounds * slots) if rounds else 1.0

    t64 = math.ceil(M / 64) * math.ceil(N / 64)
    t32 = math.ceil(M / 32) * math.ceil(N / 64)
    if fill(t32) > 1.1 * fill(t64):
        return "TL3"
    return "TL1" if t64 < slots else "TL2"


def grad_bounds(p, G, f64=True, terms=6):
    """Componentwise bounds of dA, dB, dC0 (each in its stored orientation)
    for the gradient of <G, alpha op(A) op(B) + beta C0>:
      d op(A) = conj(alpha) G op(B)^H   (contraction over N, alpha in the epilogue)
      d op(B) = op(A)^H conj(alpha) G   (contraction over M, conj(alpha) scales G
                                         as it is staged: 5 more roundings)
      dC0 = conj(beta) G                (one Hamilton product)."""
    M, N, K = p["M"], p["N"], p["K"]
    a1 = norm1(op_logical(p["opA"], p["A"], M, K))
    b1 = norm1(op_logical(p["opB"], p["B"], K, N))
    g1 = norm1(logical(G, M, N))
    al1, be1 = qnorm1(p["alpha"]), qnorm1(p["beta"])
    SdA, SdB = mag_sum(g1, b1.T), mag_sum(a1.T, g1)
    if f64:
        bA, bB, bC = bound_f64(SdA, N, al1), bound_f64(SdB, M, al1, extra=13), gamma(6, U64) * be1 * g1
    else:
        bA = bound_split(SdA, N, terms, al1)
        bB = bound_split(SdB, M, terms, al1, pre=5)
        bC = gamma(6, U_ACC32) * be1 * g1
    return (bA if p["opA"] in "NR" else bA.T), (bB if p["opB"] in "NR" else bB.T), bC
