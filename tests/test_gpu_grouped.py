"""GPU checks of the grouped (batched) FP32 path: every problem against the
FP64 oracle (relative Frobenius bar 1e-6 for 6 and 9 products, 3e-5 for 3,
globally and per 32 x 32 block, and every real within the split path's
componentwise bound), every tile class, graph capture and replay."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import SPLIT_BAR, assert_parity, dev, host, logical, relfro, split_error_bound

pytestmark = pytest.mark.gpu


def make_set(count, lo, hi, seed, opA="N", opB="N"):
    mnk = W.grouped_sizes(count, lo, hi, seed)
    g = W.rng(seed + 5)
    probs = []
    for (M, N, K) in mnk:
        M, N, K = int(M), int(N), int(K)
        ra, ca = W.stored_dims(opA, M, K)
        rb, cb = W.stored_dims(opB, K, N)
        probs.append(dict(M=M, N=N, K=K, lda=ra, ldb=rb, ldc=M,
                          A=W.qmatrix(g, ra, ca, dist="uniform", dtype=np.float32),
                          B=W.qmatrix(g, rb, cb, dist="uniform", dtype=np.float32),
                          C=W.qmatrix(g, M, N, dist="uniform", dtype=np.float32)))
    return probs


def to_dev(probs):
    return [dict(pr, A=dev(pr["A"]), B=dev(pr["B"]), C=dev(pr["C"])) for pr in probs]


def check_all(probs, dprobs, opA, opB, alpha, beta, terms=6):
    """Every problem against the oracle; returns the worst global error, the
    largest error-to-bound ratio and the worst block error."""
    worst = [0.0, 0.0, 0.0]
    for i, (pr, dp) in enumerate(zip(probs, dprobs)):
        M, N = pr["M"], pr["N"]
        want = oracle.qgemm(opA, opB, M, N, pr["K"], alpha, pr["A"], pr["lda"], pr["B"], pr["ldb"],
                            beta, pr["C"], pr["ldc"])
        p = dict(pr, opA=opA, opB=opB, alpha=alpha, beta=beta)
        st = assert_parity(logical(host(dp["C"]), M, N), logical(want, M, N), split_error_bound(p, terms),
                           SPLIT_BAR[terms], label=f"problem {i} ({M}x{N}x{pr['K']})", verbose=False)
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
