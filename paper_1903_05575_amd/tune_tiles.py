"""Tile tuner of the grouped split-BF16 kernel (FP32 plans).

The tile table maps each size class -- M and N buckets {1-16, 17-32, 33-64,
65+} and K buckets {1-64, 65+} -- to one of the four tile classes of the
grouped kernel.  The paper tuned its blocking parameters on the machine with
a search over the real kernel's run time (Sec. 5, caching parameters found
with an autotuner); this tuner does the same for the deployed objective: the
run time of ONE grouped launch over the whole batched workload (4096 problems
with M, N, K log-uniform in [8, 512], op N/N, alpha = 1, beta = 0.5).

Search: coordinate descent from the table in effect.  For every cell (in
order of the workload's flops in it) each other tile class is tried with the
rest of the table fixed; a change is kept only if the whole launch is faster
by more than `--margin` over interleaved repeats (candidate and incumbent
timed alternately, median of `--pairs` pairs of `--reps` launches each), in
two independent comparisons (the second confirms the first: single
comparisons of the whole launch differ by about 0.5% between repeats, more
than most one-cell changes are worth).  Passes repeat until one changes
nothing (or `--passes` is reached).

The table is installed at run time through qgemm_batched_set_tile_table, so
the library is not rebuilt between candidates.  The result is written as
csrc/tile_table.inc together with the launch times and a hash of the kernel
sources it was tuned on (rebuild the library after running); bench.py
reports whether the compiled table was tuned on the current kernel sources.

    python -m paper_1903_05575_amd.tune_tiles [--out PATH] [--passes 3]
"""
import argparse
import hashlib
import os
import re
import sys
import time

import numpy as np
import torch

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
# the sources whose code decides the grouped kernel's speed (not the table itself)
KERNEL_SOURCES = ("qgemm_grouped.hip", "qgemm_bf16x3_tile.hpp", "qgemm_internal.hpp", "qgemm_device.hpp")
MN_EDGES = (16, 32, 64)
K_EDGE = 64


def code_only(text):
    """Source text without comments and with whitespace runs collapsed, so that
    an edit of a comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha():
    """Hash of the code (not the comments) of the sources the grouped kernel
    is built from, excluding the table itself."""
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        h.update(code_only(open(os.path.join(CSRC, n)).read()).encode())
    return h.hexdigest()[:16]


def cell_of(M, N, K):
    bm = sum(M > e for e in MN_EDGES)
    bn = sum(N > e for e in MN_EDGES)
    bk = int(K > K_EDGE)
    return (bm * 4 + bn) * 2 + bk


def workload(count=4096, lo=8, hi=512, seed=1903055750 + 3):
    """The batched workload's sizes (log-uniform in [lo, hi], the generator of
    the benchmark) with uniform[-1, 1) operands made on the device."""
    g = np.random.default_rng(seed)
    mnk = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), (count, 3)))).astype(np.int64)
    gen = torch.Generator(device="cuda").manual_seed(1903)
    probs = []
    for M, N, K in mnk:
        M, N, K = int(M), int(N), int(K)
        mk = lambda r, c: torch.rand((c, r, 4), device="cuda", generator=gen) * 2 - 1
        probs.append(dict(M=M, N=N, K=K, lda=M, ldb=K, ldc=M, A=mk(M, K), B=mk(K, N), C=mk(M, N)))
    return probs


def launch_time(probs, table, reps, alpha=(1.0, 0.0, 0.0, 0.0), beta=(0.5, 0.0, 0.0, 0.0)):
    """One measurement: ms per launch over `reps` back-to-back launches of a
    plan built with `table` (after one warm-up launch)."""
    _lib.set_tile_table(table)
    plan = _lib.GroupedPlan(probs, "N", "N", alpha, beta)
    plan.run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    plan.close()
    return e0.elapsed_time(e1) / reps


def compare(probs, cand, inc, pairs, reps):
    """Interleaved medians (candidate, incumbent) in ms per launch."""
    tc, ti = [], []
    for _ in range(pairs):
        tc.append(launch_time(probs, cand, reps))
        ti.append(launch_time(probs, inc, reps))
    return float(np.median(tc)), float(np.median(ti))


def tune(probs, start, passes, margin, pairs, reps, log=print):
    table = list(start)
    nclass = len(_lib.TILE_CLASSES)
    flops = np.zeros(32)
    for pr in probs:
        flops[cell_of(pr["M"], pr["N"], pr["K"])] += 32.0 * pr["M"] * pr["N"] * pr["K"]
    order = [c for c in np.argsort(-flops) if flops[c] > 0]
    history = []
    t_start = compare(probs, table, table, pairs, reps)[1]
    log(f"start: {t_start:.4f} ms per launch")
    for ps in range(passes):
        changed = 0
        for cell in order:
            for cls in range(nclass):
                if cls == table[cell]:
                    continue
                cand = list(table)
                cand[cell] = cls
                tc, ti = compare(probs, cand, table, pairs, reps)
                keep = tc < ti * (1.0 - margin)
                if keep:                                 # confirm on a fresh comparison
                    tc2, ti2 = compare(probs, cand, table, pairs, reps)
                    keep = tc2 < ti2 * (1.0 - margin)
                    tc, ti = (tc + tc2) / 2, (ti + ti2) / 2
                line = (f"pass {ps + 1} cell {cell_name(cell)} class {table[cell]} -> {cls}: "
                        f"{ti:.4f} -> {tc:.4f} ms {'kept' if keep else ''}")
                log(line)
                if keep:
                    history.append(line)
                    table = cand
                    changed += 1
        if not changed:
            break
    t_end = compare(probs, table, list(start), 2 * pairs, reps)
    log(f"end: {t_end[0]:.4f} ms per launch (start table {t_end[1]:.4f} ms)")
    return table, history, t_start, t_end


def cell_name(cell):
    names = ("1-16", "17-32", "33-64", "65+")
    bm, rem = divmod(cell, 8)
    bn, bk = divmod(rem, 2)
    return f"M {names[bm]} N {names[bn]} K {'1-64' if bk == 0 else '65+'}"


def write_table(path, table, history, t_end, sha, count):
    cls = " ".join(f"{c} = {bm}x{bn}," for c, (bm, bn) in enumerate(_lib.TILE_CLASSES)).rstrip(",")
    with open(path, "w") as f:
        f.write("// Tile class per size class of the grouped split-BF16 kernel.\n")
        f.write("// Index: [M bucket][N bucket][K bucket] with M, N buckets\n")
        f.write("// {1-16, 17-32, 33-64, 65+} and K buckets {1-64, 65+}.\n")
        f.write(f"// Classes: {cls} quaternions.\n")
        f.write("// Written by paper_1903_05575_amd/tune_tiles.py: coordinate descent over the\n")
        f.write(f"// cells on the run time of one grouped launch over {count} problems (M, N, K\n")
        f.write("// log-uniform in [8, 512], op N/N); a change was kept only when the whole\n")
        f.write("// launch got faster over interleaved repeats.\n")
        f.write(f"// kernel_source_sha: {sha}\n")
        f.write(f"// launch: {t_end[1]:.4f} ms with the table tuning started from, {t_end[0]:.4f} ms with this one\n")
        for h in history:
            f.write(f"//   {h}\n")
        f.write("static const unsigned char kTileTable[4][4][2] = {\n")
        for i in range(4):
            f.write("    {" + ", ".join("{%d, %d}" % (table[(i * 4 + j) * 2], table[(i * 4 + j) * 2 + 1])
                                        for j in range(4)) + "},\n")
        f.write("};\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(CSRC, "tile_table.inc"))
    ap.add_argument("--passes", type=int, default=3)
    ap.add_argument("--margin", type=float, default=0.01)
    ap.add_argument("--pairs", type=int, default=5)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--problems", type=int, default=4096)
    args = ap.parse_args()
    if not torch.cuda.is_available():
        sys.exit("the tile tuner needs a GPU")
    _lib.lib()
    sha = kernel_source_sha()
    t0 = time.time()
    probs = workload(args.problems)
    start = _lib.tile_table()
    log = lambda s: print(s, flush=True)
    table, history, _, t_end = tune(probs, start, args.passes, args.margin, args.pairs, args.reps, log)
    _lib.set_tile_table(None)
    write_table(args.out, table, history, t_end, sha, args.problems)
    print(f"wrote {args.out} ({time.time() - t0:.0f} s); rebuild the library", flush=True)


if __name__ == "__main__":
    main()
