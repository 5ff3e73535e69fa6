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
  variants      -- the split-BF16 FP32 path, the grouped batched launch and the
                   linear-layer forward + backward, each with its own rate and
                   its error against the oracle on sampled outputs.
Other modes (used to produce the committed profiles):
    python bench.py --calibrate-copy    one 1 GiB device copy, for counter scaling
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(*names):
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(CSRC, n), "rb").read())
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


def time_launches(fn, steps, warmup):
    """Warm up, then time exactly `steps` calls.  Returns (wall ms per step,
    event ms per step on the launch stream)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
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
    return {"value": round(q.flops(M, ncols, K) / dt / 1e12, 6), "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"op {p['opA']}/{p['opB']}, M=K={M}, first {ncols} of {p['N']} columns of C "
                      f"({q.flops(M, ncols, K):.3g} flops in {dt:.1f} s)"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this library has no "
              "multi-GPU path: run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    q.lib()
    if args.calibrate_copy:
        calibrate_copy()
        return

    n = args.size
    log(f"[bench] generating FP64 {n}^3 N/N inputs")
    p = W.gemm_sweep(n, "N", "N")
    A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
    torch.cuda.synchronize()

    def step():
        q.qgemm_d("N", "N", n, n, n, p["alpha"], A, n, B, n, p["beta"], C, n)

    log(f"[bench] timing {args.steps} steps after {args.warmup} warmup")
    wall_ms, ev_ms = time_launches(step, args.steps, args.warmup)
    fl = q.flops(n, n, n)
    value = fl / (wall_ms * 1e-3) / 1e12
    achieved = fl / (ev_ms * 1e-3) / 1e12
    sha = source_sha("qgemm_f64.hip", "qgemm_internal.hpp")
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
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4),
                     "traffic": traffic, "kernel": "qgemm_f64_kernel<false,false>",
                     "kernel_ms": round(ev_ms, 3)},
    }
    del A, B, C
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle
        # size the column sample for about 15 s of oracle time on this host
        probe_cols = max(8, oracle.max_threads())
        t0 = time.perf_counter()
        cpu_baseline(p, probe_cols)
        per_col = (time.perf_counter() - t0) / probe_cols
        ncols = int(min(n, max(probe_cols, 15.0 / max(per_col, 1e-6))))
        ncols -= ncols % probe_cols if ncols > probe_cols else 0
        log(f"[bench] CPU oracle baseline on {ncols} columns")
        line["cpu_baseline"] = cpu_baseline(p, ncols)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
