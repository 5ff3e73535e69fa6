"""GPU checks of the grouped (batched) paths.  FP32 plans: every problem
against the FP64 oracle (relative Frobenius bar 1e-6 for 6 and 9 products,
3e-5 for 3, globally and per 32 x 32 block, and every real within the split
path's componentwise bound), every tile class, graph capture and replay.
FP64 plans: every problem against the oracle at the FP64 bar (1e-13) and the
FP64 componentwise bound, ragged and degenerate problems, graph replay."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import (F64_BAR, SPLIT_BAR, assert_parity, dev, error_bound, host, logical, relfro,
                            split_error_bound)

pytestmark = pytest.mark.gpu


def make_set(count, lo, hi, seed, opA="N", opB="N", dtype=np.float32):
    mnk = W.grouped_sizes(count, lo, hi, seed)
    g = W.rng(seed + 5)
    probs = []
    for (M, N, K) in mnk:
        M, N, K = int(M), int(N), int(K)
        ra, ca = W.stored_dims(opA, M, K)
        rb, cb = W.stored_dims(opB, K, N)
        probs.append(dict(M=M, N=N, K=K, lda=ra, ldb=rb, ldc=M,
                          A=W.qmatrix(g, ra, ca, dist="uniform", dtype=dtype),
                          B=W.qmatrix(g, rb, cb, dist="uniform", dtype=dtype),
                          C=W.qmatrix(g, M, N, dist="uniform", dtype=dtype)))
    return probs


def to_dev(probs):
    return [dict(pr, A=dev(pr["A"]), B=dev(pr["B"]), C=dev(pr["C"])) for pr in probs]


def check_all(probs, dprobs, opA, opB, alpha, beta, terms=6, f64=False):
    """Every problem against the oracle (split-path or FP64 bounds); returns
    the worst global error, the largest error-to-bound ratio and the worst
    block error."""
    worst = [0.0, 0.0, 0.0]
    for i, (pr, dp) in enumerate(zip(probs, dprobs)):
        M, N = pr["M"], pr["N"]
        want = oracle.qgemm(opA, opB, M, N, pr["K"], alpha, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            beta, pr["C"], pr["ldc"])
        p = dict(pr, opA=opA, opB=opB, alpha=alpha, beta=beta)
        bound, bar = (error_bound(p), F64_BAR) if f64 else (split_error_bound(p, terms), SPLIT_BAR[terms])
        st = assert_parity(logical(host(dp["C"]), M, N), logical(want, M, N), bound, bar,
                           label=f"problem {i} ({M}x{N}x{pr['K']})", verbose=False)
        worst = [max(a, b) for a, b in zip(worst, st)]
    print(f"worst over {len(probs)} problems: rel err {worst[0]:.3e}, error / componentwise bound {worst[1]:.3e}, "
          f"block rel err {worst[2]:.3e}")
    return worst[0]


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "T"), ("T", "R")])
def test_grouped_small(gpu, opA, opB):
    probs = make_set(150, 1, 150, 7 + len(opA + opB), opA, opB)
    al, be = np.array([0.6, -0.2, 0.3, 0.1]), np.array([0.5, 0.1, -0.2, 0.3])
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, opA, opB, al, be)
    plan.run()
    worst = check_all(probs, dprobs, opA, opB, al, be)
    print(f"grouped {opA}{opB}: worst rel err {worst:.2e}, {plan.info()}")
    plan.close()


@pytest.mark.parametrize("terms", [3, 9])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "C")])
def test_grouped_split_terms(gpu, terms, opA, opB):
    """The 3- and 9-product variants of the grouped kernel, each problem
    against the oracle at the single-GEMM bars."""
    probs = make_set(150, 1, 200, 200 + terms + len(opA + opB), opA, opB)
    al, be = np.array([0.6, -0.2, 0.3, 0.1]), np.array([0.5, 0.1, -0.2, 0.3])
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, opA, opB, al, be, split_terms=terms)
    plan.run()
    check_all(probs, dprobs, opA, opB, al, be, terms)
    plan.close()


@pytest.mark.parametrize("cls", range(len(q.TILE_CLASSES)))
def test_grouped_tile_classes(gpu, cls):
    probs = make_set(40, 1, 200, 100 + cls)
    al, be = np.array([1.0, 0, 0, 0]), np.array([0.5, 0, 0, 0])
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, "N", "N", al, be, tile_class=cls)
    assert plan.info()["tiles_per_class"][cls] == plan.info()["work_items"]
    plan.run()
    check_all(probs, dprobs, "N", "N", al, be)


def test_grouped_empty_and_degenerate(gpu):
    """Problems with M, N or K = 0 mixed with ordinary ones."""
    probs = make_set(10, 1, 40, 3)
    probs[2] = dict(probs[2], K=0)
    probs[5] = dict(probs[5], M=0, ldc=1, lda=1, C=probs[5]["C"])
    probs[7] = dict(probs[7], N=0)
    al, be = np.array([1.0, 0, 0, 0]), np.array([0.5, 0, 0, 0])
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, "N", "N", al, be)
    plan.run()
    for i, (pr, dp) in enumerate(zip(probs, dprobs)):
        if pr["M"] == 0 or pr["N"] == 0:
            np.testing.assert_array_equal(host(dp["C"]), pr["C"])
            continue
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], al, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            be, pr["C"], pr["ldc"])
        p = dict(pr, opA="N", opB="N", alpha=al, beta=be)
        assert_parity(logical(host(dp["C"]), pr["M"], pr["N"]), logical(want, pr["M"], pr["N"]),
                      split_error_bound(p), 1e-6, label=f"degenerate set, problem {i}")
    q.GroupedPlan([], "N", "N", al, be).run()


def test_grouped_graph_replay(gpu):
    """The run captured in a graph: each replay (with eager work and syncs in
    between) equals the eager run bit for bit."""
    probs = make_set(60, 1, 130, 11)
    al, be = np.array([1.0, 0, 0, 0]), np.array([0.5, 0, 0, 0])
    eager = to_dev(probs)
    plan_e = q.GroupedPlan(eager, "N", "N", al, be)
    graphd = to_dev(probs)
    plan_g = q.GroupedPlan(graphd, "N", "N", al, be)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan_g.run()
    # capture does not execute: graph buffers still hold the inputs
    for dp, pr in zip(graphd, probs):
        np.testing.assert_array_equal(host(dp["C"]), pr["C"])
    for rep in range(3):
        plan_e.run()
        g.replay()
        junk = torch.randn(1000, device="cuda") * 2      # unrelated eager work between replays
        torch.cuda.synchronize()
        del junk
        for a, b in zip(eager, graphd):
            np.testing.assert_array_equal(host(a["C"]), host(b["C"]))
    plan_e.close()
    plan_g.close()


@pytest.mark.slow
def test_grouped_4096_all_problems(gpu):
    """4096 problems, M, N, K log-uniform in [8, 512], op N/N, alpha = 1,
    beta = 0.5: every problem against the oracle."""
    w = W.grouped()
    probs = w["problems"]
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, "N", "N", w["alpha"], w["beta"])
    plan.run()
    worst = check_all(probs, dprobs, "N", "N", w["alpha"], w["beta"])
    print(f"grouped 4096: worst rel err {worst:.2e}, {plan.info()}")


F64_OPS = [("N", "N"), ("C", "T"), ("T", "R"), ("R", "C")]


@pytest.mark.parametrize("opA,opB", F64_OPS)
def test_grouped_f64(gpu, opA, opB):
    """An FP64 plan of 160 problems, M, N, K log-uniform in [1, 300] (many
    ragged tiles), quaternion alpha and beta: every problem against the
    oracle at the FP64 bar and componentwise bound."""
    probs = make_set(160, 1, 300, 300 + len(opA + opB) + ord(opA[0]), opA, opB, dtype=np.float64)
    al, be = np.array([0.6, -0.2, 0.3, 0.1]), np.array([0.5, 0.1, -0.2, 0.3])
    dprobs = to_dev(probs)
    plan = q.GroupedPlan(dprobs, opA, opB, al, be, dtype=torch.float64)
    info = plan.info()
    assert info["tiles_per_class"][0] == info["work_items"]
    plan.run()
    worst = check_all(probs, dprobs, opA, opB, al, be, f64=True)
    print(f"grouped FP64 {opA}{opB}: worst rel err {worst:.2e}, {info}")
    plan.close()


def test_grouped_f64_degenerate(gpu):
    """FP64 plan with M, N or K = 0 beside ordinary problems, and a second
    plan with alpha = 0 whose A and B hold NaN (never read: C <- beta C) and
    one with beta = 0 whose C holds NaN (never read)."""
    probs = make_set(12, 1, 70, 21, dtype=np.float64)
    probs[2] = dict(probs[2], K=0)
    probs[5] = dict(probs[5], M=0, ldc=1, lda=1)
    probs[7] = dict(probs[7], N=0)
    al, be = np.array([0.6, -0.2, 0.3, 0.1]), np.array([0.5, 0.1, -0.2, 0.3])
    dprobs = to_dev(probs)
    q.GroupedPlan(dprobs, "N", "N", al, be, dtype=torch.float64).run()
    for i, (pr, dp) in enumerate(zip(probs, dprobs)):
        if pr["M"] == 0 or pr["N"] == 0:
            np.testing.assert_array_equal(host(dp["C"]), pr["C"])
            continue
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], al, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            be, pr["C"], pr["ldc"])
        p = dict(pr, opA="N", opB="N", alpha=al, beta=be)
        assert_parity(logical(host(dp["C"]), pr["M"], pr["N"]), logical(want, pr["M"], pr["N"]),
                      error_bound(p), F64_BAR, label=f"FP64 degenerate set, problem {i}")
    zero = np.zeros(4)
    nan_ab = [dict(pr, A=np.full_like(pr["A"], np.nan), B=np.full_like(pr["B"], np.nan)) for pr in probs]
    d2 = to_dev(nan_ab)
    q.GroupedPlan(d2, "N", "N", zero, be, dtype=torch.float64).run()
    for i, (pr, dp) in enumerate(zip(nan_ab, d2)):
        if pr["M"] == 0 or pr["N"] == 0:
            continue
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], zero, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            be, pr["C"], pr["ldc"])
        np.testing.assert_allclose(logical(host(dp["C"]), pr["M"], pr["N"]), logical(want, pr["M"], pr["N"]),
                                   rtol=1e-15, atol=1e-15, err_msg=f"alpha = 0, problem {i}")
    nan_c = [dict(pr, C=np.full_like(pr["C"], np.nan)) for pr in probs]
    d3 = to_dev(nan_c)
    q.GroupedPlan(d3, "N", "N", al, zero, dtype=torch.float64).run()
    for i, (pr, dp) in enumerate(zip(nan_c, d3)):
        if pr["M"] == 0 or pr["N"] == 0:
            continue
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], al, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            zero, pr["C"], pr["ldc"])
        p = dict(pr, opA="N", opB="N", alpha=al, beta=zero)
        assert_parity(logical(host(dp["C"]), pr["M"], pr["N"]), logical(want, pr["M"], pr["N"]),
                      error_bound(p), F64_BAR, label=f"FP64 beta = 0, problem {i}")


def test_grouped_f64_graph_replay(gpu):
    """An FP64 plan captured in a graph: each replay (with eager work and
    syncs in between) equals the eager run bit for bit, and the first equals
    the oracle."""
    probs = make_set(150, 1, 200, 31, "T", "C", dtype=np.float64)
    al, be = np.array([0.3, 0.2, -0.4, 0.5]), np.array([0.5, -0.1, 0.2, 0.05])
    eager = to_dev(probs)
    plan_e = q.GroupedPlan(eager, "T", "C", al, be, dtype=torch.float64)
    graphd = to_dev(probs)
    plan_g = q.GroupedPlan(graphd, "T", "C", al, be, dtype=torch.float64)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan_g.run()
    for dp, pr in zip(graphd, probs):
        np.testing.assert_array_equal(host(dp["C"]), pr["C"])
    for rep in range(3):
        plan_e.run()
        g.replay()
        junk = torch.randn(1000, device="cuda") * 2      # unrelated eager work between replays
        torch.cuda.synchronize()
        del junk
        for a, b in zip(eager, graphd):
            np.testing.assert_array_equal(host(a["C"]), host(b["C"]))
        if rep == 0:
            check_all(probs, graphd, "T", "C", al, be, f64=True)
    plan_e.close()
    plan_g.close()


def test_grouped_f64_matches_single(gpu):
    """Every problem of an FP64 plan equals qgemm_d on the same problem bit
    for bit (the same tile arithmetic in the same order)."""
    probs = make_set(60, 1, 260, 41, "C", "N", dtype=np.float64)
    al, be = np.array([0.3, 0.2, -0.4, 0.5]), np.array([0.5, -0.1, 0.2, 0.05])
    grouped = to_dev(probs)
    q.GroupedPlan(grouped, "C", "N", al, be, dtype=torch.float64).run()
    for i, (pr, dp) in enumerate(zip(probs, grouped)):
        C = dev(pr["C"])
        q.qgemm_d("C", "N", pr["M"], pr["N"], pr["K"], al, dev(pr["A"]), pr["lda"], dev(pr["B"]), pr["ldb"], be,
                  C, pr["ldc"])
        np.testing.assert_array_equal(host(dp["C"]), host(C), err_msg=f"problem {i}")


def test_grouped_runtime_tile_table(gpu):
    """A table installed at run time (the tuner's hook) decides the classes of
    plans created afterwards, and their results stay within the bounds; a plan
    made before the change keeps its own classes."""
    import paper_1903_05575_amd._lib as lb
    probs = make_set(60, 1, 200, 61)
    al, be = np.array([0.6, -0.2, 0.3, 0.1]), np.array([0.5, 0.1, -0.2, 0.3])
    d_before = to_dev(probs)
    before = q.GroupedPlan(d_before, "N", "N", al, be)
    counts_before = before.info()["tiles_per_class"]
    try:
        for cls in range(len(q.TILE_CLASSES)):
            lb.set_tile_table([cls] * 32)
            dprobs = to_dev(probs)
            plan = q.GroupedPlan(dprobs, "N", "N", al, be)
            info = plan.info()
            assert info["tiles_per_class"][cls] == info["work_items"], (cls, info)
            plan.run()
            check_all(probs, dprobs, "N", "N", al, be)
            plan.close()
    finally:
        lb.set_tile_table(None)
    assert before.info()["tiles_per_class"] == counts_before
    before.run()
    check_all(probs, d_before, "N", "N", al, be)
    before.close()
