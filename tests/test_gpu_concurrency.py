"""Calls from several host threads, each on its own stream, run concurrently
and give the same bits as the same calls made one after another (the
library keeps no shared mutable state beyond the once-per-device kernel
attributes; the kernels are deterministic)."""
import threading

import numpy as np
import pytest
import torch

import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def jobs():
    """Independent work items: (name, make_buffers, call(bufs))."""
    out = []
    p = W.gemm_problem(1700, 700, 650, 300, "N", "C", pad=1)
    out.append(("qgemm_d", lambda: {"A": dev(p["A"]), "B": dev(p["B"]), "C": dev(p["C"])},
                lambda b: q.qgemm_d("N", "C", 700, 650, 300, p["alpha"], b["A"], p["lda"], b["B"], p["ldb"], p["beta"],
                                    b["C"], p["ldc"])))
    s = W.gemm_problem(1701, 900, 500, 400, "T", "N", dtype=np.float32)
    out.append(("qgemm_s", lambda: {"A": dev(s["A"]), "B": dev(s["B"]), "C": dev(s["C"])},
                lambda b: q.qgemm_s("T", "N", 900, 500, 400, s["alpha"], b["A"], s["lda"], b["B"], s["ldb"], s["beta"],
                                    b["C"], s["ldc"])))
    g = W.rng(1702)
    A = W.qmatrix(g, 500, 300)
    C = W.qmatrix(g, 500, 500)
    out.append(("qherk_d", lambda: {"A": dev(A), "C": dev(C)},
                lambda b: q.qherk("L", "N", 500, 300, 1.0, b["A"], 500, 0.5, b["C"], 500)))
    m = W.mixed_problem(1703, "Q", "R", 400, 600, 350)
    out.append(("qgemm_mixed_d", lambda: {"A": dev(m["A"]), "B": dev(m["B"]), "C": dev(m["C"])},
                lambda b: q.qgemm_mixed("Q", "R", "N", "N", 400, 600, 350, m["alpha"], b["A"], m["lda"], b["B"],
                                        m["ldb"], m["beta"], b["C"], m["ldc"])))
    x, y = W.qvector(g, 300_000), W.qvector(g, 300_000)
    out.append(("qaxpy_d", lambda: {"x": dev(x), "y": dev(y)}, lambda b: q.qaxpy(300_000, m["alpha"], b["x"], 1, b["y"], 1)))
    return out


def test_threads_and_streams_match_sequential(gpu):
    work = jobs()
    seq = []
    for _, mk, call in work:
        b = mk()
        for _ in range(3):
            call(b)
        seq.append(b)
    torch.cuda.synchronize()
    bufs = [mk() for _, mk, _ in work]
    torch.cuda.synchronize()
    errors = []

    def worker(i):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for _ in range(3):
                    work[i][2](bufs[i])
            st.synchronize()
        except Exception as e:                    # reported in the main thread
            errors.append((work[i][0], e))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(work))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    torch.cuda.synchronize()
    for (name, _, _), a, b in zip(work, seq, bufs):
        for k in a:
            np.testing.assert_array_equal(host(a[k]), host(b[k]), err_msg=f"{name}:{k}")
