"""Benchmark of the MI355X quaternion GEMM (one JSON line on stdout).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-variants]

A step is one FP64 quaternion GEMM C <- alpha op(A) op(B) + beta C at
M = N = K = 8192, op N/N, random quaternion alpha and beta, A/B/C components
U[-1,1] (seeded, synthetic), with operands resident in HBM.  The value is the
effective throughput 32 M N K / t (16 real multiply-adds per quaternion
multiply-add, 2 flops each).  Beside it the line carries:
  roofline      -- the FP64 kernel against the MI355X FP64 matrix peak, from HIP
                   events around the timed launches on the launch stream, plus
                   HBM traffic from the committed rocprofv3 counter summary when
                   it was taken on the current kernel source;
  cpu_baseline  -- the CPU oracle timed on this host on a bounded column sample;
  variants      -- the split-BF16 FP32 path, the grouped batched launch (FP32
                   and FP64), the
                   linear-layer forward + backward, the general scalar
                   placement, the Hermitian rank-k update, the triangular
                   multiply, the mixed-type products, the level-1/2
                   operations and the one-GPU row shard, each with its own
                   rate and its error against the oracle on sampled outputs,
                   plus vendor context (rocBLAS ZGEMM / DGEMM on embeddings).
Other modes (used to produce the committed profiles):
    python bench.py --calibrate-copy    one 1 GiB device copy, for counter scaling
    python bench.py --probe-ops         one launch per op pair at 2048, for per-kernel counters
    python bench.py --only fp64|split|grouped|grouped_f64|linear|scalars|herk|trmm|mixed|blas12|shard|context
                                                   one part, no CPU baseline
    python bench.py --sweep                        FP64 sizes 1024..8192 x op pairs, one line each
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
import paper_1903_05575_amd as q  # noqa: E402

METRIC = "effective qgemm TFLOP/s (32·MNK) & % matrix peak, FP64 vs split-BF16 at stated err"
PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 matrix (published)
PEAK_BF16 = 2500.0    # TFLOP/s, MI355X dense BF16 matrix (published)
PEAK_HBM = 8000.0     # GB/s
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1903_05575_amd", "csrc")
FP64_SOURCES = ("qgemm_f64.hip", "qgemm_f64_tile.hpp", "qgemm_internal.hpp", "qgemm_device.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(*names):
    """Hash of the code (comments stripped) of the named kernel sources: a
    profile taken on other code is not reported against this one."""
    from paper_1903_05575_amd.tune_tiles import code_only
    h = hashlib.sha256()
    for n in names:
        h.update(code_only(open(os.path.join(CSRC, n)).read()).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag, sha):
    """HBM bytes per launch from profiles/<kernel_tag>_traffic.md, or None if
    absent or taken on another version of the kernel source."""
    path = os.path.join(PROFILES, f"{kernel_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_source_sha:\s*(\w+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def time_launches(fn, steps, warmup, min_ms=0.0):
    """Warm up, then time exactly `steps` calls.  Returns (wall ms per step,
    event ms per step on the launch stream).  With min_ms > 0 the warm-up is
    extended to at least min_ms of launches and the timed region to at least
    as many launches as fill min_ms: the GPU clock drops within a fraction of
    a second of idling and takes tens of milliseconds to settle under a new
    load, so a few launches of a short kernel would time the ramp."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if min_ms > 0:
        t0, n = time.perf_counter(), 0
        while (time.perf_counter() - t0) * 1e3 < min_ms:
            fn()
            n += 1
            if n % 8 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        steps = max(steps, int(np.ceil(min_ms / ((time.perf_counter() - t0) * 1e3 / n))))
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, e0.elapsed_time(e1) / steps


VARIANT_MIN_MS = 400.0


def time_variant(fn, steps, warmup):
    """time_launches for the secondary lines: at least VARIANT_MIN_MS of warm
    launches and of timed launches (the headline times exactly --steps)."""
    return time_launches(fn, steps, warmup, min_ms=VARIANT_MIN_MS)


def cpu_baseline(p, ncols):
    """Oracle on the first `ncols` columns of C (same A, alpha, beta)."""
    import oracle
    threads = oracle.max_threads()
    M, K = p["M"], p["K"]
    B = p["B"][:ncols]
    C = p["C"][:ncols]
    t0 = time.perf_counter()
    oracle.qgemm(p["opA"], p["opB"], M, ncols, K, p["alpha"], p["A"], p["lda"], B, p["ldb"],
                 p["beta"], C, p["ldc"])
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(q.flops(M, ncols, K) / dt / 1e12, 6), "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle", "host_cpu": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)),
            "sample": f"op {p['opA']}/{p['opB']}, M=K={M}, first {ncols} of {p['N']} columns of C "
                      f"({q.flops(M, ncols, K):.3g} flops in {dt:.1f} s)"}


def oracle_single_thread():
    """The oracle on one thread: the whole 64^3 op N/N problem, and 1024^3 op
    N/N on its first 32 columns of C (a few seconds)."""
    import oracle
    threads = oracle.max_threads()
    oracle.set_threads(1)
    out = {}
    try:
        for n, ncols in ((64, 64), (1024, 32)):
            p = W.gemm_problem(W.BASE_SEED + 7, n, n, n, "N", "N", dist="normal")
            reps = 20 if n == 64 else 1
            t0 = time.perf_counter()
            for _ in range(reps):
                oracle.qgemm("N", "N", n, ncols, n, p["alpha"], p["A"], p["lda"], p["B"][:ncols], p["ldb"],
                             p["beta"], p["C"][:ncols], p["ldc"])
            dt = (time.perf_counter() - t0) / reps
            out[f"{n}_cubed"] = {"gflops": round(q.flops(n, ncols, n) / dt / 1e9, 3),
                                 "columns": ncols, "seconds": round(dt, 4)}
    finally:
        oracle.set_threads(threads)
    return out


def oracle_all_cores():
    """The oracle on all host threads at M = N = K = 64, 1024, 2048 and 4096
    (op N/N): the whole 64^3 problem, and the first 128, 64 and 32 columns of
    C at the larger sizes (each column is a full M x K by K product)."""
    import oracle
    out = {}
    for n, ncols in ((64, 64), (1024, 128), (2048, 64), (4096, 32)):
        p = W.gemm_problem(W.BASE_SEED + 7, n, n, n, "N", "N", dist="normal") if n <= 1024 else \
            W.gemm_problem(W.BASE_SEED + 7, n, ncols, n, "N", "N", dist="normal")
        reps = 20 if n == 64 else 1
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.qgemm("N", "N", n, ncols, n, p["alpha"], p["A"], p["lda"], p["B"][:ncols], p["ldb"],
                         p["beta"], p["C"][:ncols], p["ldc"])
        dt = (time.perf_counter() - t0) / reps
        out[f"{n}_cubed"] = {"gflops": round(q.flops(n, ncols, n) / dt / 1e9, 3), "columns": ncols,
                             "seconds": round(dt, 4)}
    return out


def relfro(got, want):
    den = np.linalg.norm(want)
    return float(np.linalg.norm(np.asarray(got, np.float64) - want) / (den if den > 0 else 1.0))


def sampled_error(p, Cdev, nrows, ncols, seed):
    """Relative Frobenius error of a computed C (device, storage layout) against
    the oracle on a seeded nrows x ncols sample of output entries (each entry
    is the full K-term sum; the oracle computes only the sampled entries).
    Returns (error, sample description)."""
    import oracle
    g = np.random.default_rng(seed)
    rows = np.sort(g.choice(p["M"], min(nrows, p["M"]), replace=False))
    cols = np.sort(g.choice(p["N"], min(ncols, p["N"]), replace=False))
    want = oracle.qgemm_entries(p["opA"], p["opB"], p["K"], p["alpha"], p["A"], p["B"], p["beta"], p["C"],
                                rows, cols)
    got = Cdev[torch.from_numpy(cols).cuda()][:, torch.from_numpy(rows).cuda()].cpu().numpy()
    return relfro(got, want), f"{len(rows)} x {len(cols)} entries (seeded)"


def variant_split(steps, warmup):
    """FP32 4096^3 op N/C on the split-BF16 path (N(0,1) entries and the
    row-scaled case) beside the FP64 path on the same widened data; error
    against the oracle on a seeded 256 x 48 sample of C."""
    import oracle
    out = {}
    n = 4096
    fl = q.flops(n, n, n)
    for scaled in (False, True):
        p = W.gemm_precision(n, scaled=scaled)
        A, B = dev(p["A"]), dev(p["B"])
        C = torch.zeros((n, n, 4), dtype=torch.float32, device="cuda")
        wall, ev = time_variant(lambda: q.qgemm_s("N", "C", n, n, n, p["alpha"], A, n, B, n, p["beta"], C, n),
                                 steps, warmup)
        g = np.random.default_rng(11 + scaled)
        rows = np.sort(g.choice(n, 256, replace=False))
        cols = np.sort(g.choice(n, 48, replace=False))
        want = oracle.qgemm_entries("N", "C", n, p["alpha"], p["A"], p["B"], p["beta"],
                                    p["C"].astype(np.float64), rows, cols)
        got = C.cpu().numpy()[cols][:, rows]
        key = "split_bf16_4096_NC" + ("_rowscaled" if scaled else "")
        tf = fl / (ev * 1e-3) / 1e12
        out[key] = {"ms": round(ev, 3), "tflops_effective": round(tf, 2),
                    "frac_bf16_peak": round(tf / PEAK_BF16, 4),
                    "bf16_mfma_utilization": round(6 * tf / PEAK_BF16, 4), "split_terms": 6,
                    "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}
        if not scaled:
            A64, B64 = A.double(), B.double()
            C64 = torch.zeros((n, n, 4), dtype=torch.float64, device="cuda")
            wall64, ev64 = time_variant(
                lambda: q.qgemm_d("N", "C", n, n, n, p["alpha"], A64, n, B64, n, p["beta"], C64, n),
                max(1, steps // 2), 1)
            got64 = C64.cpu().numpy()[cols][:, rows]
            out["fp64_4096_NC_same_data"] = {"ms": round(ev64, 3),
                                              "tflops_effective": round(fl / (ev64 * 1e-3) / 1e12, 2),
                                              "rel_err_vs_oracle_sampled": float(f"{relfro(got64, want):.3e}")}
            out[key]["speedup_vs_fp64_path"] = round(ev64 / ev, 2)
            del A64, B64, C64
            torch.cuda.empty_cache()
            # vendor context: one BF16 product of the same real contraction, (4M x 4K) by (4K x N), as a
            # hipBLASLt GEMM through torch.matmul; the split path runs six such products
            X = torch.randn(4 * n, 4 * n, dtype=torch.bfloat16, device="cuda")
            Y = torch.randn(4 * n, n, dtype=torch.bfloat16, device="cuda")
            _, evv = time_variant(lambda: torch.matmul(X, Y), steps, warmup)
            vendor = 2.0 * (4 * n) * (4 * n) * n / (evv * 1e-3) / 1e12
            out["context_vendor_bf16_gemm_16384x4096x16384"] = {
                "ms": round(evv, 3), "tflops_bf16": round(vendor, 1),
                "frac_bf16_peak": round(vendor / PEAK_BF16, 4),
                "split_path_bf16_rate_over_vendor": round(6 * tf / vendor, 3)}
            del X, Y
        del A, B, C
        torch.cuda.empty_cache()
    return out


def variant_grouped(steps, warmup):
    """4096 FP32 problems, M, N, K log-uniform in [8, 512], op N/N, alpha = 1,
    beta = 0.5: one persistent launch replayed from a captured graph; error
    on 64 sampled problems (the first replay's output, C restored before)."""
    import oracle
    w = W.grouped()
    probs = [dict(pr, A=dev(pr["A"]), B=dev(pr["B"]), C=dev(pr["C"])) for pr in w["problems"]]
    plan = q.GroupedPlan(probs, "N", "N", w["alpha"], w["beta"])
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        plan.run()
    graph.replay()
    torch.cuda.synchronize()
    g = np.random.default_rng(3)
    sample = sorted(g.choice(len(probs), 64, replace=False))
    err = 0.0
    for i in sample:
        pr = w["problems"][i]
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], w["alpha"], pr["A"], pr["lda"], pr["B"],
                            pr["ldb"], w["beta"], pr["C"], pr["ldc"])
        err = max(err, relfro(probs[i]["C"].cpu().numpy(), want))
    wall, ev = time_variant(graph.replay, steps * 4, warmup)
    fl = sum(q.flops(pr["M"], pr["N"], pr["K"]) for pr in w["problems"])
    by = sum(16 * (pr["M"] * pr["K"] + pr["K"] * pr["N"] + 2 * pr["M"] * pr["N"]) for pr in w["problems"])
    tf = fl / (ev * 1e-3) / 1e12
    info = plan.info()
    plan.close()
    table_txt = open(os.path.join(CSRC, "tile_table.inc")).read()
    m_sha = re.search(r"kernel_source_sha:\s*(\w+)", table_txt)
    tuned_sha = m_sha.group(1) if m_sha else None
    from paper_1903_05575_amd.tune_tiles import kernel_source_sha
    kernel_sha = kernel_source_sha()
    return {"grouped_4096_fp32": {"ms": round(ev, 3), "tflops_effective": round(tf, 2),
                                  "tile_table_tuned_on_current_kernel": tuned_sha == kernel_sha,
                                  "bf16_mfma_utilization": round(6 * tf / PEAK_BF16, 4),
                                  "algorithmic_gbps": round(by / (ev * 1e-3) / 1e9, 1),
                                  "hbm_frac": round(by / (ev * 1e-3) / 1e9 / PEAK_HBM, 4),
                                  "graph_replay": True, "work_items": info["work_items"],
                                  "worst_rel_err_64_sampled_problems": float(f"{err:.3e}")}}


def variant_grouped_f64(steps, warmup):
    """The same 4096 problem sizes (M, N, K log-uniform in [8, 512], op N/N,
    alpha = 1, beta = 0.5) in FP64 as one persistent launch of the FP64 tile,
    replayed from a captured graph; error on 64 sampled problems (the first
    replay's output)."""
    import oracle
    w = W.grouped(dtype=np.float64)
    probs = [dict(pr, A=dev(pr["A"]), B=dev(pr["B"]), C=dev(pr["C"])) for pr in w["problems"]]
    plan = q.GroupedPlan(probs, "N", "N", w["alpha"], w["beta"], dtype=torch.float64)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        plan.run()
    graph.replay()
    torch.cuda.synchronize()
    g = np.random.default_rng(4)
    sample = sorted(g.choice(len(probs), 64, replace=False))
    err = 0.0
    for i in sample:
        pr = w["problems"][i]
        want = oracle.qgemm("N", "N", pr["M"], pr["N"], pr["K"], w["alpha"], pr["A"], pr["lda"], pr["B"],
                            pr["ldb"], w["beta"], pr["C"], pr["ldc"])
        err = max(err, relfro(probs[i]["C"].cpu().numpy(), want))
    wall, ev = time_variant(graph.replay, steps * 4, warmup)
    fl = sum(q.flops(pr["M"], pr["N"], pr["K"]) for pr in w["problems"])
    by = sum(32 * (pr["M"] * pr["K"] + pr["K"] * pr["N"] + 2 * pr["M"] * pr["N"]) for pr in w["problems"])
    tf = fl / (ev * 1e-3) / 1e12
    info = plan.info()
    plan.close()
    return {"grouped_4096_fp64": {"ms": round(ev, 3), "tflops_effective": round(tf, 2),
                                  "frac_fp64_peak": round(tf / PEAK_FP64, 4),
                                  "algorithmic_gbps": round(by / (ev * 1e-3) / 1e9, 1),
                                  "graph_replay": True, "work_items": info["work_items"],
                                  "worst_rel_err_64_sampled_problems": float(f"{err:.3e}")}}


def variant_grouped_kscan(steps, warmup):
    """Cost model of the FP32 batched launch: the 4096 problems' M and N with
    K forced to 16, 32, 64 and 128 (1, 2, 4, 8 K-tiles of 16 per item), and
    with their own K; time per graph replay and the item and K-tile counts
    of each plan.  The slope is the cost of one K-tile over all items, the
    intercept the per-item cost (descriptor, first K-tile, epilogue)."""
    from paper_1903_05575_amd import _lib
    from paper_1903_05575_amd.tune_tiles import cell_of
    mnk = W.grouped_sizes()
    g = W.rng(W.BASE_SEED + 40)
    out = {}
    for kfix in (None, 16, 32, 64, 128):
        probs = []
        for M, N, K in mnk:
            M, N, K = int(M), int(N), int(K) if kfix is None else kfix
            probs.append(dict(M=M, N=N, K=K, lda=M, ldb=K, ldc=M, A=dev(W.qmatrix(g, M, K, dtype=np.float32)),
                              B=dev(W.qmatrix(g, K, N, dtype=np.float32)),
                              C=torch.zeros((N, M, 4), dtype=torch.float32, device="cuda")))
        plan = q.GroupedPlan(probs, "N", "N", (1.0, 0.0, 0.0, 0.0), (0.5, 0.0, 0.0, 0.0))
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            plan.run()
        _, ev = time_variant(graph.replay, steps * 4, warmup)
        info = plan.info()
        plan.close()
        # K-tiles walked: ceil(K / 16) per item of the problem (every class walks K-tiles of 16)
        table = _lib.tile_table()
        ktiles = 0
        for pr in probs:
            cell = cell_of(pr["M"], pr["N"], pr["K"])
            bm, bn = _lib.TILE_CLASSES[table[cell]]
            ktiles += -(-pr["M"] // bm) * -(-pr["N"] // bn) * -(-pr["K"] // 16)
        out["K=" + ("own" if kfix is None else str(kfix))] = {"ms": round(ev, 4), "work_items": info["work_items"],
                                                               "k_tiles": ktiles}
        del probs, graph
        torch.cuda.empty_cache()
    return {"grouped_4096_fp32_k_scan": out}


def variant_linear(steps, warmup):
    """Quaternion linear layer Y = X W, X 8192 x 1024, W 1024 x 1024 (FP32,
    Glorot), forward + hand-written backward (dX, dW) through torch.autograd;
    error on sampled rows of Y and dX against the oracle."""
    import oracle
    p = W.linear_layer()
    M, K, N = p["M"], p["K"], p["N"]
    X = dev(p["X"]).requires_grad_(True)
    layer = q.QLinear(K, N)
    with torch.no_grad():
        layer.weight.copy_(dev(p["W"]))
    dY = dev(p["dY"])

    def fwd():
        return layer(X)

    def fwd_bwd():
        X.grad = None
        layer.weight.grad = None
        layer(X).backward(dY)

    _, ev_f = time_variant(fwd, steps, warmup)
    _, ev_fb = time_variant(fwd_bwd, steps, warmup)
    Y = fwd().detach().cpu().numpy()
    fwd_bwd()
    dX = X.grad.cpu().numpy()
    g = np.random.default_rng(5)
    rows = np.sort(g.choice(M, 32, replace=False))
    one, zero = np.array([1.0, 0, 0, 0]), np.zeros(4)
    Xs = p["X"][:, rows, :].astype(np.float64)
    Wd = p["W"].astype(np.float64)
    Ys = oracle.qgemm("N", "N", 32, N, K, one, Xs, 32, Wd, K, zero, np.zeros((N, 32, 4)), 32)
    dXs, _, _ = oracle.qgemm_backward("N", "N", 32, N, K, one, Xs, 32, Wd, K,
                                      p["dY"][:, rows, :].astype(np.float64), 32, zero,
                                      want_dB=False, want_dC0=False)
    fl = 3 * q.flops(M, N, K)
    return {"linear_8192x1024x1024_fp32": {
        "forward_ms": round(ev_f, 3), "forward_backward_ms": round(ev_fb, 3),
        "tflops_effective_fwd_bwd": round(fl / (ev_fb * 1e-3) / 1e12, 2),
        "rel_err_Y_sampled": float(f"{relfro(Y[:, rows], Ys):.3e}"),
        "rel_err_dX_sampled": float(f"{relfro(dX[:, rows], dXs):.3e}")}}


def variant_scalars(steps, warmup):
    """General scalar placement (qgemm_ex_d): FP64 4096^3 N/N with left, middle
    and right alpha and left and right beta, beside qgemm_d on the same data;
    error on a 64 x 32 sample against the oracle's qgemm_ex."""
    import oracle
    n = 4096
    p = W.gemm_problem(W.BASE_SEED + 5, n, n, n, "N", "N")
    g = W.rng(W.BASE_SEED + 6)
    aL, aM, aR, bL, bR = (g.uniform(-1, 1, 4) for _ in range(5))
    A, B = dev(p["A"]), dev(p["B"])
    C0 = dev(p["C"])
    C = C0.clone()
    _, ev = time_variant(lambda: q.qgemm_ex("N", "N", n, n, n, aL, aM, aR, A, n, B, n, bL, bR, C, n), steps, warmup)
    C2 = C0.clone()
    _, ev_d = time_variant(lambda: q.qgemm_d("N", "N", n, n, n, aL, A, n, B, n, bL, C2, n), steps, warmup)
    C.copy_(C0)
    q.qgemm_ex("N", "N", n, n, n, aL, aM, aR, A, n, B, n, bL, bR, C, n)
    gs = np.random.default_rng(7)
    rows = np.sort(gs.choice(n, 64, replace=False))
    cols = np.sort(gs.choice(n, 32, replace=False))
    Bs = np.ascontiguousarray(p["B"][cols])
    Cs = np.ascontiguousarray(p["C"][cols][:, rows])
    As = np.ascontiguousarray(p["A"][:, rows])
    want = oracle.qgemm_ex("N", "N", 64, 32, n, aL, aM, aR, As, 64, Bs, n, bL, bR, Cs, 64)
    got = C.cpu().numpy()[cols][:, rows]
    fl = q.flops(n, n, n)
    return {"fp64_ex_4096_all_scalars": {"ms": round(ev, 3), "tflops_effective": round(fl / (ev * 1e-3) / 1e12, 2),
                                         "qgemm_d_same_data_ms": round(ev_d, 3),
                                         "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}}


def variant_herk(steps, warmup):
    """Hermitian rank-k update qherk_d: lower triangle of C <- alpha A A^H + beta C,
    N = K = 8192 FP64 (alpha = 1, beta = 0.5); effective flops 32 K N (N + 1) / 2;
    error on sampled lower-triangle entries against the oracle."""
    import oracle
    n = 8192
    g = W.rng(W.BASE_SEED + 7)
    A = W.qmatrix(g, n, n, dist="uniform")
    C = W.qmatrix(g, n, n, dist="uniform")
    Ad, Cd0 = dev(A), dev(C)
    Cd = Cd0.clone()
    _, ev = time_variant(lambda: q.qherk("L", "N", n, n, 1.0, Ad, n, 0.5, Cd, n), steps, warmup)
    Cd.copy_(Cd0)
    q.qherk("L", "N", n, n, 1.0, Ad, n, 0.5, Cd, n)
    gs = np.random.default_rng(8)
    cols = np.sort(gs.choice(n // 2, 16, replace=False))
    rows = np.sort(gs.choice(np.arange(n // 2 + 1, n), 64, replace=False))   # strictly below the diagonal
    want = oracle.qgemm_entries("N", "C", n, np.array([1.0, 0, 0, 0]), A, A, np.array([0.5, 0, 0, 0]), C, rows, cols)
    got = Cd.cpu().numpy()[cols][:, rows]
    fl = 32 * n * n * (n + 1) // 2
    return {"fp64_herk_8192_lower": {"ms": round(ev, 3), "tflops_effective": round(fl / (ev * 1e-3) / 1e12, 2),
                                     "frac_fp64_peak": round(fl / (ev * 1e-3) / 1e12 / PEAK_FP64, 4),
                                     "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}}


def variant_trmm(steps, warmup):
    """Triangular multiply qtrmm_d: C <- alpha L B with L the lower triangle of
    A (side left, op N, non-unit diagonal), M = N = 8192 FP64; the upper
    triangle of A holds NaN (never read).  Effective flops 32 N M (M + 1) / 2;
    error on 16 whole columns against the oracle's qtrmm."""
    import oracle
    n = 8192
    t = W.trmm_problem(W.BASE_SEED + 8, "L", "L", "N", "N", n, n)
    Ad, Bd = dev(t["A"]), dev(t["B"])
    Cd = torch.empty_like(Bd)
    al = t["alpha"]
    _, ev = time_variant(lambda: q.qtrmm("L", "L", "N", "N", n, n, al, Ad, n, Bd, n, Cd, n), steps, warmup)
    gs = np.random.default_rng(9)
    cols = np.sort(gs.choice(n, 16, replace=False))
    Bs = np.ascontiguousarray(t["B"][cols])
    want = oracle.qtrmm("L", "L", "N", "N", n, 16, al, t["A"], n, Bs, n, np.zeros_like(Bs), n)
    got = Cd.cpu().numpy()[cols]
    fl = 32 * n * n * (n + 1) // 2
    return {"fp64_trmm_8192_left_lower": {"ms": round(ev, 3), "tflops_effective": round(fl / (ev * 1e-3) / 1e12, 2),
                                          "frac_fp64_peak": round(fl / (ev * 1e-3) / 1e12 / PEAK_FP64, 4),
                                          "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}}


def variant_mixed(steps, warmup):
    """Mixed-type GEMM qgemm_mixed_d, FP64 M = N = K = 8192 op N/N: quaternion
    x real (4 real multiply-adds per element product, 8 MNK flops) and complex
    x quaternion (8 multiply-adds, 16 MNK flops), and quaternion x real with
    float storage (qgemm_mixed_s, FP64 products); error on a 64 x 32 sample
    against the oracle's qgemm_mixed on the same stored inputs."""
    import oracle
    n = 8192
    out = {}
    for tA, tB, fpm, name, dt in (("Q", "R", 8, "fp64_mixed_8192_quat_x_real", np.float64),
                                  ("Z", "Q", 16, "fp64_mixed_8192_complex_x_quat", np.float64),
                                  ("Q", "R", 8, "fp32_storage_mixed_8192_quat_x_real", np.float32)):
        p = W.mixed_problem(W.BASE_SEED + 9 + fpm, tA, tB, n, n, n)
        p = dict(p, A=p["A"].astype(dt), B=p["B"].astype(dt), C=p["C"].astype(dt))
        A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
        C0 = C.clone()
        _, ev = time_variant(lambda: q.qgemm_mixed(tA, tB, "N", "N", n, n, n, p["alpha"], A, n, B, n, p["beta"], C, n),
                              steps, warmup)
        C.copy_(C0)
        q.qgemm_mixed(tA, tB, "N", "N", n, n, n, p["alpha"], A, n, B, n, p["beta"], C, n)
        gs = np.random.default_rng(10)
        rows = np.sort(gs.choice(n, 64, replace=False))
        cols = np.sort(gs.choice(n, 32, replace=False))
        As = np.ascontiguousarray(p["A"][:, rows])
        Bs = np.ascontiguousarray(p["B"][cols])
        Cs = np.ascontiguousarray(p["C"][cols][:, rows])
        want = oracle.qgemm_mixed(tA, tB, "N", "N", 64, 32, n, p["alpha"], As, 64, Bs, n, p["beta"], Cs, 64)
        got = C.cpu().numpy()[cols][:, rows]
        fl = fpm * n * n * n
        out[name] = {"ms": round(ev, 3), "tflops_useful": round(fl / (ev * 1e-3) / 1e12, 2),
                     "frac_fp64_peak": round(fl / (ev * 1e-3) / 1e12 / PEAK_FP64, 4),
                     "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}
        del A, B, C, C0
        torch.cuda.empty_cache()
    return out


def variant_blas12(steps, warmup):
    """Level-1/2 operations, HBM-bound: algorithmic bytes (each operand read
    once, each output written once) over the HIP-event time, against the
    8 TB/s HBM peak.  gemv 8192 x 8192 FP64 (op N and op C) and FP32 (op N),
    axpy and dotc over 2^26 FP64 quaternions; errors against the oracle.
    These calls take well under a millisecond, so each is timed over ten
    times the requested number of steps."""
    import oracle
    steps = 10 * steps
    out = {}
    g = W.rng(W.BASE_SEED + 20)
    M = N = 8192
    A64 = W.qmatrix(g, M, N)
    x64, y64 = W.qvector(g, N), W.qvector(g, M)
    al, be = W.quaternion(g), W.quaternion(g)
    for trans, dt, name in (("N", np.float64, "fp64_gemv_8192_N"), ("C", np.float64, "fp64_gemv_8192_C"),
                            ("N", np.float32, "fp32_gemv_8192_N")):
        A, x, y = dev(A64.astype(dt)), dev(x64.astype(dt)), dev(y64.astype(dt))
        y0 = y.clone()
        _, ev = time_variant(lambda: q.qgemv(trans, M, N, al, A, M, x, 1, be, y, 1), steps, warmup)
        y.copy_(y0)
        q.qgemv(trans, M, N, al, A, M, x, 1, be, y, 1)
        want = oracle.qgemv(trans, M, N, al, A64.astype(dt), M, x64.astype(dt), 1, be, y64.astype(dt), 1)
        es = np.dtype(dt).itemsize * 4
        nbytes = es * (M * N + N + 2 * M)
        out[name] = {"ms": round(ev, 4), "algorithmic_gbps": round(nbytes / (ev * 1e-3) / 1e9, 1),
                     "hbm_frac": round(nbytes / (ev * 1e-3) / 8e12, 4),
                     "rel_err_vs_oracle": float(f"{relfro(y.cpu().numpy(), want):.3e}")}
        del A, x, y, y0
    n = 1 << 26
    xs, ys = W.qvector(g, n), W.qvector(g, n)
    x, y = dev(xs), dev(ys)
    y0 = y.clone()
    _, ev = time_variant(lambda: q.qaxpy(n, al, x, 1, y, 1), steps, warmup)
    y.copy_(y0)
    q.qaxpy(n, al, x, 1, y, 1)
    sl = slice(0, 1 << 16)
    want = oracle.qaxpy(1 << 16, al, xs[sl], 1, ys[sl], 1)
    out["fp64_axpy_2^26"] = {"ms": round(ev, 4), "algorithmic_gbps": round(96 * n / (ev * 1e-3) / 1e9, 1),
                             "hbm_frac": round(96 * n / (ev * 1e-3) / 8e12, 4),
                             "rel_err_vs_oracle_first_65536": float(f"{relfro(y.cpu().numpy()[sl], want):.3e}")}
    res = torch.empty(4, dtype=torch.float64, device="cuda")
    work = torch.empty(q._lib.DOT_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    _, ev = time_variant(lambda: q.qdot(n, x, 1, y0, 1, conj=True, result=res, work=work), steps, warmup)
    want = oracle.qdot(True, n, xs, 1, ys, 1)
    out["fp64_dotc_2^26"] = {"ms": round(ev, 4), "algorithmic_gbps": round(64 * n / (ev * 1e-3) / 1e9, 1),
                             "hbm_frac": round(64 * n / (ev * 1e-3) / 8e12, 4),
                             "rel_err_vs_oracle": float(f"{relfro(res.cpu().numpy(), want):.3e}")}
    # achievable-bandwidth reference: a plain device copy of the same 2^26 quaternions
    _, ev = time_variant(lambda: y0.copy_(x), steps, warmup)
    out["reference_device_copy_2^26"] = {"ms": round(ev, 4), "gbps": round(64 * n / (ev * 1e-3) / 1e9, 1),
                                         "hbm_frac": round(64 * n / (ev * 1e-3) / 8e12, 4)}
    del x, y, y0
    torch.cuda.empty_cache()
    return out


def variant_shard(steps, warmup):
    """One GPU's share of an 8-way row split of the 8192^3 FP64 GEMM:
    M = 1024 rows of op(A) and C, N = K = 8192 (op N/N)."""
    M, N, K = 1024, 8192, 8192
    p = W.gemm_problem(W.BASE_SEED + 30, M, N, K, "N", "N")
    A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
    _, ev = time_variant(lambda: q.qgemm_d("N", "N", M, N, K, p["alpha"], A, M, B, K, p["beta"], C, M), steps,
                          warmup)
    fl = q.flops(M, N, K)
    return {"fp64_row_shard_1024x8192x8192": {"ms": round(ev, 3), "tflops_effective": round(fl / (ev * 1e-3) / 1e12, 2),
                                              "frac_fp64_peak": round(fl / (ev * 1e-3) / 1e12 / PEAK_FP64, 4)}}


def variant_context(steps, warmup):
    """Vendor context for the 8192^3 FP64 product on the same data (not a
    target): rocBLAS ZGEMM through torch.matmul on the complex block
    representation [[A0 + i A1, A2 + i A3], [-conj(A2 + i A3), conj(A0 + i A1)]]
    (2M x 2K times 2K x 2N, 64 MNK real flops), and rocBLAS DGEMM on the real
    left-multiplication embedding L(op A) (4M x 4K) times B read as a 4K x N
    real matrix (32 MNK flops, the same contraction this library runs)."""
    import oracle
    n = 8192
    p = W.gemm_sweep(n, "N", "N")
    one, zero = np.array([1.0, 0, 0, 0]), np.zeros(4)
    out = {}
    A = dev(p["A"])                       # storage (K, M, 4): A[k, m, c]
    B = dev(p["B"])                       # storage (N, K, 4)
    with torch.no_grad():
        def cblock(S):                    # logical (rows, cols) from storage (cols, rows, 4)
            z0 = torch.complex(S[..., 0], S[..., 1]).T
            z1 = torch.complex(S[..., 2], S[..., 3]).T
            return torch.cat([torch.cat([z0, z1], 1), torch.cat([-z1.conj(), z0.conj()], 1)], 0).contiguous()
        Ac, Bc = cblock(A), cblock(B)
        _, ev = time_variant(lambda: torch.matmul(Ac, Bc), steps, warmup)
        Cc = torch.matmul(Ac, Bc)
        rows, cols = np.arange(0, n, n // 16), np.arange(3, n, n // 16)
        want = oracle.qgemm_entries("N", "N", n, one, p["A"], p["B"], zero, p["C"], rows, cols)   # (cols, rows, 4)
        top0 = Cc[:n, :n][rows][:, cols].cpu().numpy().T
        top1 = Cc[:n, n:][rows][:, cols].cpu().numpy().T
        got = np.stack([top0.real, top0.imag, top1.real, top1.imag], -1)
        out["context_rocblas_zgemm_block_embedding_8192"] = {
            "ms": round(ev, 3), "tflops_zgemm_counted": round(64 * n ** 3 / (ev * 1e-3) / 1e12, 2),
            "tflops_quaternion_effective": round(32 * n ** 3 / (ev * 1e-3) / 1e12, 2),
            "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}
        del Ac, Bc, Cc
        torch.cuda.empty_cache()
        # L(a)[r][c] = sign(r, c) a[r ^ c], rows 4 mu + r, columns 4 k + c
        sign = torch.tensor([[1, -1, -1, -1], [1, 1, -1, 1], [1, 1, 1, -1], [1, -1, 1, 1]], dtype=torch.float64,
                            device="cuda")
        idx = torch.tensor([[r ^ c for c in range(4)] for r in range(4)], device="cuda")
        Al = A.permute(1, 0, 2)           # (M, K, 4)
        AL = (Al[:, :, idx] * sign).permute(0, 2, 1, 3).reshape(4 * n, 4 * n).contiguous()   # (M, r, K, c)
        Br = B.reshape(n, 4 * n).T.contiguous()                                           # (4K, N)
        del Al
        _, ev = time_variant(lambda: torch.matmul(AL, Br), steps, warmup)
        Cr = torch.matmul(AL, Br).reshape(n, 4, n)                                       # (M, r, N)
        got = Cr[rows][:, :, cols].permute(2, 0, 1).cpu().numpy()                         # (cols, rows, 4)
        out["context_rocblas_dgemm_L_embedding_8192"] = {
            "ms": round(ev, 3), "tflops_effective": round(32 * n ** 3 / (ev * 1e-3) / 1e12, 2),
            "rel_err_vs_oracle_sampled": float(f"{relfro(got, want):.3e}")}
        del AL, Br, Cr
    del A, B
    torch.cuda.empty_cache()
    return out


def sweep(steps, warmup):
    """FP64 qgemm_d over M = N = K in 1024..8192 and every op pair of N, T, C:
    one JSON line per case (event time per launch, effective TFLOP/s and the
    relative Frobenius error of one launch's output against the oracle on a
    seeded sample of entries: all of C at 1024, 256 x 128 entries above);
    every case is timed over at least 0.4 s of launches after 0.4 s of warm
    launches, and sizes up to 2048 in three such windows of which the median
    is reported (a one-off clock change would otherwise decide the figure)."""
    import oracle
    for n in W.SWEEP_SIZES:
        for opA, opB in W.OP_PAIRS:
            p = W.gemm_sweep(n, opA, opB)
            A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
            C0 = C.clone()
            # short launches need more of them for steady clocks
            st, wu, win = (max(steps, 50), max(warmup, 10), 3) if n <= 2048 else (steps, warmup, 1)
            evs = [time_variant(lambda: q.qgemm_d(opA, opB, n, n, n, p["alpha"], A, p["lda"], B, p["ldb"],
                                                   p["beta"], C, p["ldc"]), st, wu)[1] for _ in range(win)]
            ev = sorted(evs)[len(evs) // 2]
            C.copy_(C0)                                   # one launch on the pristine C, checked
            q.qgemm_d(opA, opB, n, n, n, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], C, p["ldc"])
            torch.cuda.synchronize()
            if n <= 1024:
                want = oracle.qgemm(opA, opB, n, n, n, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"], p["beta"],
                                    p["C"], p["ldc"])
                err, sample = relfro(C.cpu().numpy(), want), "all entries"
            else:
                err, sample = sampled_error(p, C, 256, 128, seed=n + 7 * W.OP_PAIRS.index((opA, opB)))
            fl = q.flops(n, n, n)
            print(json.dumps({"sweep": f"{n} {opA}/{opB}", "ms": round(ev, 3),
                              "tflops_effective": round(fl / (ev * 1e-3) / 1e12, 2),
                              "frac_fp64_peak": round(fl / (ev * 1e-3) / 1e12 / PEAK_FP64, 4),
                              "rel_err_vs_oracle": float(f"{err:.3e}"), "err_sample": sample}), flush=True)
            del A, B, C, C0
            torch.cuda.empty_cache()


def probe_ops(n=2048):
    """One launch per op pair of qgemm_d (at M = N = K = n and n / 2, whose
    grid takes the 32 x 32 tiles) and qgemm_s (at n), of qgemm_mixed_d for each
    type pair (op N/N and T/T) at n, and of qgemm_mixed_s for the real type
    pairs: a short program for per-kernel counter runs (LDS bank conflicts by
    op pair)."""
    widths = {"R": 1, "Z": 2, "Q": 4}
    for dt, fn, m in ((torch.float64, q.qgemm_d, n), (torch.float64, q.qgemm_d, n // 2),
                      (torch.float32, q.qgemm_s, n)):
        A = torch.rand(m * m * 4, dtype=dt, device="cuda")
        B = torch.rand(m * m * 4, dtype=dt, device="cuda")
        C = torch.zeros(m * m * 4, dtype=dt, device="cuda")
        for oa, ob in W.OP_PAIRS:
            fn(oa, ob, m, m, m, (1, 0, 0, 0), A, m, B, m, (0, 0, 0, 0), C, m)
            torch.cuda.synchronize()
            log(f"{'qgemm_d' if dt == torch.float64 else 'qgemm_s'} {oa}/{ob} n={m}")
    for ta, tb in (("Q", "R"), ("R", "Q"), ("Z", "Q"), ("Q", "Z")):
        for oa, ob in (("N", "N"), ("T", "T")):
            A = torch.rand(n * n * widths[ta], dtype=torch.float64, device="cuda")
            B = torch.rand(n * n * widths[tb], dtype=torch.float64, device="cuda")
            C = torch.zeros(n * n * 4, dtype=torch.float64, device="cuda")
            q.qgemm_mixed(ta, tb, oa, ob, n, n, n, (1, 0, 0, 0), A, n, B, n, (0, 0, 0, 0), C, n)
            torch.cuda.synchronize()
            log(f"qgemm_mixed {ta}x{tb} {oa}/{ob} n={n}")
    # float storage: a real operand takes the 32 x 64 tiles with 8-kappa K-tiles there
    for ta, tb in (("Q", "R"), ("R", "Q")):
        for oa, ob in (("N", "N"), ("T", "T")):
            A = torch.rand(n * n * widths[ta], dtype=torch.float32, device="cuda")
            B = torch.rand(n * n * widths[tb], dtype=torch.float32, device="cuda")
            C = torch.zeros(n * n * 4, dtype=torch.float32, device="cuda")
            q.qgemm_mixed(ta, tb, oa, ob, n, n, n, (1, 0, 0, 0), A, n, B, n, (0, 0, 0, 0), C, n)
            torch.cuda.synchronize()
            log(f"qgemm_mixed_s {ta}x{tb} {oa}/{ob} n={n}")


def smi_reading():
    """Socket power (W), GFX clock (MHz) and the board power cap (W) as the
    system management tools report them now (None where they report none)."""
    import subprocess
    out = {"socket_power_w": None, "gfx_clk_mhz": None, "power_cap_w": None}
    try:
        r = subprocess.run(["amd-smi", "metric", "--json"], capture_output=True, text=True, timeout=30)
        d, _ = json.JSONDecoder().raw_decode(r.stdout[r.stdout.index("{"):])
        g = d["gpu_data"][0] if "gpu_data" in d else d[0]
        out["socket_power_w"] = g["power"]["socket_power"]["value"]
        out["gfx_clk_mhz"] = g["clock"]["gfx_0"]["clk"]["value"]
    except (OSError, ValueError, KeyError, IndexError, TypeError, subprocess.SubprocessError):
        pass
    try:
        r = subprocess.run(["rocm-smi", "-M", "--json"], capture_output=True, text=True, timeout=30)
        d, _ = json.JSONDecoder().raw_decode(r.stdout[r.stdout.index("{"):])
        out["power_cap_w"] = float(next(iter(d.values()))["Max Graphics Package Power (W)"])
    except (OSError, ValueError, KeyError, StopIteration, TypeError, subprocess.SubprocessError):
        pass
    return out


def power_probe(seconds=12.0):
    """Each of four kernels kept busy for `seconds` of back-to-back launches:
    FP64 qgemm_d at 8192^3 N/N, the split-BF16 qgemm_s at 4096^3 N/C, the
    vendor BF16 GEMM (hipBLASLt through torch.matmul) on one product of the
    split path's real contraction (16384 x 16384 by 16384 x 4096), and the
    4096-problem FP32 batched launch (graph replays).  Half-way through, the
    socket power and GFX clock are read from amd-smi; one JSON line per
    kernel with the sustained rate beside them."""
    import threading
    n64, n32 = 8192, 4096
    cases = []
    p = W.gemm_sweep(n64, "N", "N")
    A64, B64, C64 = dev(p["A"]), dev(p["B"]), dev(p["C"])
    cases.append(("qgemm_d 8192^3 N/N (FP64 MFMA)", q.flops(n64, n64, n64), "TFLOP/s effective",
                  lambda: q.qgemm_d("N", "N", n64, n64, n64, p["alpha"], A64, n64, B64, n64, p["beta"], C64, n64)))
    ps = W.gemm_precision(n32)
    A32, B32 = dev(ps["A"]), dev(ps["B"])
    C32 = torch.zeros((n32, n32, 4), dtype=torch.float32, device="cuda")
    cases.append(("qgemm_s 4096^3 N/C (split BF16, 6 products)", q.flops(n32, n32, n32), "TFLOP/s effective",
                  lambda: q.qgemm_s("N", "C", n32, n32, n32, ps["alpha"], A32, n32, B32, n32, ps["beta"], C32, n32)))
    X = torch.randn(4 * n32, 4 * n32, dtype=torch.bfloat16, device="cuda")
    Y = torch.randn(4 * n32, n32, dtype=torch.bfloat16, device="cuda")
    cases.append(("vendor BF16 GEMM 16384x16384 by 16384x4096", 2.0 * (4 * n32) ** 2 * n32, "TFLOP/s BF16",
                  lambda: torch.matmul(X, Y)))
    w = W.grouped()
    probs = [dict(pr, A=dev(pr["A"]), B=dev(pr["B"]), C=dev(pr["C"])) for pr in w["problems"]]
    plan = q.GroupedPlan(probs, "N", "N", w["alpha"], w["beta"])
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        plan.run()
    cases.append(("batched FP32, 4096 problems (split BF16, 6 products)",
                  sum(q.flops(pr["M"], pr["N"], pr["K"]) for pr in w["problems"]), "TFLOP/s effective",
                  graph.replay))
    for name, fl, unit, fn in cases:
        fn()
        torch.cuda.synchronize()
        reading = {}
        th = threading.Timer(seconds / 2, lambda: reading.update(smi_reading()))
        t0, cnt = time.perf_counter(), 0
        th.start()
        while time.perf_counter() - t0 < seconds:
            for _ in range(4):
                fn()
            torch.cuda.synchronize()
            cnt += 4
        dt = time.perf_counter() - t0
        th.join()
        rate = fl * cnt / dt / 1e12
        line = {"power": name, "launches": cnt, "ms": round(dt / cnt * 1e3, 3), "rate": round(rate, 1),
                "unit": unit, **reading}
        # matrix-core work: six BF16 products per effective flop on the split paths (tile padding not counted)
        line["matrix_tflops"] = round(rate * (6 if "6 products" in name else 1), 1)
        if reading.get("socket_power_w"):
            line["matrix_tflops_per_w"] = round(line["matrix_tflops"] / reading["socket_power_w"], 3)
        print(json.dumps(line), flush=True)
    plan.close()


def calibrate_copy():
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    x.fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log(f"copied {n} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--power", action="store_true",
                    help="sustained rate, socket power and clock of the FP64, split, vendor BF16 and batched GEMMs")
    ap.add_argument("--probe-ops", action="store_true", help="one launch per op pair at 2048 (for counter runs)")
    ap.add_argument("--sweep", action="store_true", help="time the FP64 size x op-pair sweep, one line per case")
    ap.add_argument("--only", choices=["fp64", "split", "grouped", "grouped_f64", "grouped_kscan", "linear", "scalars",
                                       "herk", "trmm", "mixed", "blas12", "shard", "context"],
                    help="run one part only and print its figures (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this library has no "
              "multi-GPU path: run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    q.lib()
    if args.power:
        power_probe()
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.probe_ops:
        probe_ops()
        return
    if args.sweep:
        sweep(args.steps, args.warmup)
        return

    if args.only in ("split", "grouped", "grouped_f64", "grouped_kscan", "linear", "scalars", "herk", "trmm",
                     "mixed", "blas12", "shard", "context"):
        fn = {"split": variant_split, "grouped": variant_grouped, "grouped_f64": variant_grouped_f64,
              "grouped_kscan": variant_grouped_kscan,
              "linear": variant_linear,
              "scalars": variant_scalars, "herk": variant_herk, "trmm": variant_trmm,
              "mixed": variant_mixed, "blas12": variant_blas12, "shard": variant_shard,
              "context": variant_context}[args.only]
        print(json.dumps(fn(args.steps, args.warmup)), flush=True)
        return

    n = args.size
    log(f"[bench] generating FP64 {n}^3 N/N inputs")
    p = W.gemm_sweep(n, "N", "N")
    A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
    torch.cuda.synchronize()

    def step():
        q.qgemm_d("N", "N", n, n, n, p["alpha"], A, n, B, n, p["beta"], C, n)

    C0 = C.clone()
    log(f"[bench] timing {args.steps} steps after {args.warmup} warmup")
    wall_ms, ev_ms = time_launches(step, args.steps, args.warmup)
    # after the timed region: one launch on the pristine C, checked against the oracle on sampled entries
    C.copy_(C0)
    step()
    torch.cuda.synchronize()
    del C0
    log("[bench] checking the timed launch's output against the oracle")
    head_err, head_sample = sampled_error(p, C, 256, 128, seed=8192)
    fl = q.flops(n, n, n)
    value = fl / (wall_ms * 1e-3) / 1e12
    achieved = fl / (ev_ms * 1e-3) / 1e12
    sha = source_sha(*FP64_SOURCES)
    traffic = read_traffic(f"qgemm_f64_{n}", sha)
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 quaternion GEMM M=N=K={n}, op N/N, lda=M, random quaternion "
                               "alpha/beta, A/B/C components U[-1,1] (seeded)",
                   "M": n, "N": n, "K": n, "opA": "N", "opB": "N",
                   "pct_of_fp64_matrix_peak": round(100 * value / PEAK_FP64, 2)},
        "rel_err_vs_oracle_sampled": float(f"{head_err:.3e}"),
        "err_sample": f"{head_sample} of C from one launch of the timed kernel on the same inputs",
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4),
                     "traffic": traffic, "kernel": "qgemm_f64_kernel<32,false,false,false,0,64>",
                     "kernel_ms": round(ev_ms, 3)},
    }
    del A, B, C
    torch.cuda.empty_cache()
    if args.only == "fp64":
        print(json.dumps(line), flush=True)
        return
    if not args.no_variants:
        variants = {}
        for name, fn in (("split", variant_split), ("grouped", variant_grouped),
                         ("grouped_f64", variant_grouped_f64), ("linear", variant_linear),
                         ("scalars", variant_scalars), ("herk", variant_herk), ("trmm", variant_trmm),
                         ("mixed", variant_mixed), ("blas12", variant_blas12), ("shard", variant_shard),
                         ("context", variant_context)):
            log(f"[bench] variant {name}")
            variants.update(fn(args.steps, args.warmup))
            torch.cuda.empty_cache()
        line["variants"] = variants
    if not args.no_cpu_baseline:
        import oracle
        # size the column sample for about 20 s of oracle time on this host
        probe_cols = max(8, oracle.max_threads())
        t0 = time.perf_counter()
        cpu_baseline(p, probe_cols)
        per_col = (time.perf_counter() - t0) / probe_cols
        ncols = int(min(n, max(probe_cols, 20.0 / max(per_col, 1e-6))))
        ncols -= ncols % probe_cols if ncols > probe_cols else 0
        log(f"[bench] CPU oracle baseline on {ncols} columns")
        line["cpu_baseline"] = cpu_baseline(p, ncols)
        line["cpu_baseline"]["single_thread"] = oracle_single_thread()
        line["cpu_baseline"]["all_cores_by_size"] = oracle_all_cores()
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
