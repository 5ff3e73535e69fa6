"""Every entry point captured into a HIP graph: the library launches kernels
only (no allocation, copy or synchronisation), so a captured call replays.
Each graph is replayed three times with unrelated eager work and a
synchronisation in between, and after every replay its buffers must equal,
bit for bit, those of the same call made eagerly the same number of times."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def replay_matches(make_buffers, call):
    """make_buffers() -> dict of device tensors (fresh copies of the same
    inputs); call(bufs) enqueues the operation on the current stream."""
    eager, graphed = make_buffers(), make_buffers()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        call(graphed)
    for rep in range(3):
        call(eager)
        g.replay()
        junk = torch.randn(4096, device="cuda") * 3       # unrelated eager work
        torch.cuda.synchronize()
        del junk
        for k in eager:
            np.testing.assert_array_equal(host(eager[k]), host(graphed[k]), err_msg=f"{k} after replay {rep}")


def test_graph_qgemm_d_s_ex(gpu):
    p = W.gemm_problem(1400, 130, 90, 70, "N", "C", pad=1)
    for dtype in (torch.float64, torch.float32):
        mk = lambda: {"A": dev(p["A"], dtype), "B": dev(p["B"], dtype), "C": dev(p["C"], dtype)}
        if dtype == torch.float64:
            fn = lambda b: q.qgemm_d("N", "C", 130, 90, 70, p["alpha"], b["A"], p["lda"], b["B"], p["ldb"],
                                     p["beta"], b["C"], p["ldc"])
        else:
            fn = lambda b: q.qgemm_s("N", "C", 130, 90, 70, p["alpha"], b["A"], p["lda"], b["B"], p["ldb"],
                                     p["beta"], b["C"], p["ldc"])
        replay_matches(mk, fn)
    mk = lambda: {"A": dev(p["A"]), "B": dev(p["B"]), "C": dev(p["C"])}
    sc = W.rng(1401).uniform(-1, 1, (3, 4))
    replay_matches(mk, lambda b: q.qgemm_ex("N", "C", 130, 90, 70, p["alpha"], sc[0], sc[1], b["A"], p["lda"],
                                            b["B"], p["ldb"], p["beta"], sc[2], b["C"], p["ldc"]))


def test_graph_herk_trmm_mixed(gpu):
    g = W.rng(1410)
    A = W.qmatrix(g, 100, 60)
    C = W.qmatrix(g, 100, 100)
    replay_matches(lambda: {"A": dev(A), "C": dev(C)},
                   lambda b: q.qherk("U", "N", 100, 60, 0.5, b["A"], 100, 0.9, b["C"], 100))
    t = W.trmm_problem(1411, "R", "L", "C", "U", 80, 110)
    replay_matches(lambda: {"A": dev(t["A"]), "B": dev(t["B"]), "C": dev(np.zeros_like(t["C"]))},
                   lambda b: q.qtrmm("R", "L", "C", "U", 80, 110, t["alpha"], b["A"], t["lda"], b["B"], t["ldb"],
                                     b["C"], t["ldc"]))
    m = W.mixed_problem(1412, "Z", "Q", 70, 90, 50, "T", "N")
    replay_matches(lambda: {"A": dev(m["A"]), "B": dev(m["B"]), "C": dev(m["C"])},
                   lambda b: q.qgemm_mixed("Z", "Q", "T", "N", 70, 90, 50, m["alpha"], b["A"], m["lda"], b["B"],
                                           m["ldb"], m["beta"], b["C"], m["ldc"]))


def test_graph_level12(gpu):
    g = W.rng(1420)
    n = 50_000
    x, y = W.qvector(g, n), W.qvector(g, n)
    al, be = W.quaternion(g), W.quaternion(g)
    replay_matches(lambda: {"x": dev(x), "y": dev(y)}, lambda b: q.qaxpy(n, al, b["x"], 1, b["y"], 1))
    replay_matches(lambda: {"x": dev(x), "y": dev(y), "r": dev(np.zeros(4)),
                            "w": torch.zeros(q._lib.DOT_WORK_DOUBLES, dtype=torch.float64, device="cuda")},
                   lambda b: q.qdot(n, b["x"], 1, b["y"], 1, conj=True, result=b["r"], work=b["w"]))
    A = W.qmatrix(g, 300, 200)
    xv, yv = W.qvector(g, 300), W.qvector(g, 200)
    replay_matches(lambda: {"A": dev(A), "x": dev(xv), "y": dev(yv)},
                   lambda b: q.qgemv("C", 300, 200, al, b["A"], 300, b["x"], 1, be, b["y"], 1))


def test_graph_backward(gpu):
    p = W.gemm_problem(1430, 60, 50, 40, "T", "N")
    G = W.qmatrix(W.rng(1431), 60, 50)
    mk = lambda: {"A": dev(p["A"]), "B": dev(p["B"]), "G": dev(G), "dA": dev(np.zeros_like(p["A"])),
                  "dB": dev(np.zeros_like(p["B"])), "dC0": dev(np.zeros_like(G))}
    replay_matches(mk, lambda b: q.qgemm_backward("T", "N", 60, 50, 40, p["alpha"], b["A"], p["lda"], b["B"],
                                                  p["ldb"], b["G"], 60, p["beta"], b["dA"], p["lda"], b["dB"],
                                                  p["ldb"], b["dC0"], 60))
