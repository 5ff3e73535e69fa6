"""Tile tuner of the grouped split-BF16 kernel.

For every size class of the tile table -- M and N buckets {8-16, 17-32,
33-64, 65-512} and K buckets {8-64, 65-512} -- it builds a synthetic group of
problems with sizes drawn log-uniformly inside the class, times one grouped
launch with each tile class forced, and keeps the fastest.
The result is written as csrc/tile_table.inc (the table compiled into
libqgemm.so; rebuild after running) together with the measured times.

    python -m paper_1903_05575_amd.tune_tiles [--out PATH] [--problems 256]
"""
import argparse
import math
import os
import sys

import torch

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
MN_BUCKETS = ((8, 16), (17, 32), (33, 64), (65, 512))
K_BUCKETS = ((8, 64), (65, 512))


def make_group(count, mb, nb, kb, gen):
    probs = []
    for _ in range(count):
        def draw(lo, hi):
            u = torch.rand((), generator=gen).item()
            return int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
        M, N, K = draw(*mb), draw(*nb), draw(*kb)
        A = torch.rand((K, M, 4), device="cuda") * 2 - 1
        B = torch.rand((N, K, 4), device="cuda") * 2 - 1
        C = torch.rand((N, M, 4), device="cuda") * 2 - 1
        probs.append(dict(M=M, N=N, K=K, lda=M, ldb=K, ldc=M, A=A, B=B, C=C))
    return probs


def time_plan(plan, reps=5):
    plan.run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(count, log=print):
    gen = torch.Generator().manual_seed(1903)
    table = [[[0, 0] for _ in MN_BUCKETS] for _ in MN_BUCKETS]
    notes = []
    one, half = (1.0, 0.0, 0.0, 0.0), (0.5, 0.0, 0.0, 0.0)
    for i, mb in enumerate(MN_BUCKETS):
        for j, nb in enumerate(MN_BUCKETS):
            for k, kb in enumerate(K_BUCKETS):
                probs = make_group(count, mb, nb, kb, gen)
                times = []
                for cls in range(len(_lib.TILE_CLASSES)):
                    plan = _lib.GroupedPlan(probs, "N", "N", one, half, tile_class=cls)
                    times.append(time_plan(plan))
                    plan.close()
                best = min(range(len(times)), key=lambda c: times[c])
                table[i][j][k] = best
                line = (f"M {mb[0]}-{mb[1]} N {nb[0]}-{nb[1]} K {kb[0]}-{kb[1]}: "
                        + " ".join(f"{t:.3f}" for t in times) + f" ms -> class {best}")
                notes.append(line)
                log(line)
                del probs
    return table, notes


def write_table(path, table, notes, count):
    cls = " ".join(f"{c} = {bm}x{bn}," for c, (bm, bn) in enumerate(_lib.TILE_CLASSES)).rstrip(",")
    with open(path, "w") as f:
        f.write("// Tile class per size class of the grouped split-BF16 kernel.\n")
        f.write("// Index: [M bucket][N bucket][K bucket] with M, N buckets\n")
        f.write("// {1-16, 17-32, 33-64, 65+} and K buckets {1-64, 65+}.\n")
        f.write(f"// Classes: {cls} quaternions.\n")
        f.write("// Written by paper_1903_05575_amd/tune_tiles.py: fastest class of one grouped\n")
        f.write(f"// launch over {count} problems drawn log-uniformly inside each size class\n")
        f.write(f"// (times in ms for classes 0..{len(_lib.TILE_CLASSES) - 1}):\n")
        for n in notes:
            f.write(f"//   {n}\n")
        f.write("static const unsigned char kTileTable[4][4][2] = {\n")
        for i in range(4):
            f.write("    {" + ", ".join("{%d, %d}" % tuple(table[i][j]) for j in range(4)) + "},\n")
        f.write("};\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tile_table.inc"))
    ap.add_argument("--problems", type=int, default=256)
    args = ap.parse_args()
    if not torch.cuda.is_available():
        sys.exit("the tile tuner needs a GPU")
    _lib.lib()
    table, notes = tune(args.problems, log=lambda s: print(s, flush=True))
    write_table(args.out, table, notes, args.problems)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
