"""Host logic of the tile tuner (no GPU): its size classes agree with the
library's, the table file it writes round-trips through the library's
run-time table, and the committed table was tuned on the current kernel
sources (the hash it records matches)."""
import os
import re


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cell_of_matches_bucket_edges():
    from paper_1903_05575_amd import tune_tiles as t
    # M, N buckets 1-16, 17-32, 33-64, 65+; K buckets 1-64, 65+ (include/qgemm.h)
    def bucket(x):
        return 0 if x <= 16 else 1 if x <= 32 else 2 if x <= 64 else 3
    for M in (1, 16, 17, 32, 33, 64, 65, 512):
        for N in (1, 16, 17, 32, 33, 64, 65, 512):
            for K in (1, 64, 65, 512):
                assert t.cell_of(M, N, K) == (bucket(M) * 4 + bucket(N)) * 2 + int(K > 64)
    names = {t.cell_name(c) for c in range(32)}
    assert len(names) == 32


def test_written_table_round_trips(tmp_path):
    """write_table's text, compiled into kTileTable order, is what
    qgemm_batched_set_tile_table takes and qgemm_batched_get_tile_table returns."""
    from paper_1903_05575_amd import tune_tiles as t
    import paper_1903_05575_amd._lib as lb
    table = [(3 * c + 1) % 4 for c in range(32)]
    path = tmp_path / "tile_table.inc"
    t.write_table(str(path), table, ["pass 1 cell M 1-16 N 1-16 K 1-64 class 0 -> 1: 1.0 -> 0.9 ms kept"],
                  (0.9, 1.0), "0123456789abcdef", 4096)
    txt = path.read_text()
    body = txt[txt.index("kTileTable"):]
    vals = [int(v) for v in re.findall(r"\b(\d)\b", body[body.index("=") + 1:])]
    assert vals == table
    lb.set_tile_table(vals)
    try:
        assert lb.tile_table() == table
    finally:
        lb.set_tile_table(None)
    assert "kernel_source_sha: 0123456789abcdef" in txt


def test_committed_table_tuned_on_current_kernel():
    from paper_1903_05575_amd import tune_tiles as t
    txt = open(os.path.join(ROOT, "paper_1903_05575_amd", "csrc", "tile_table.inc")).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]{16})", txt)
    assert m, "tile_table.inc carries no kernel hash"
    assert m.group(1) == t.kernel_source_sha(), \
        "the grouped kernel sources changed since the table was tuned: re-run tune_tiles on a GPU"
