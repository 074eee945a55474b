"""Host logic of bench.py (no GPU): the algorithmic bytes the roofline is
priced on, the layout read back from a profiled run's log, and the gates
that keep a committed counter profile out of the bench line once the
kernels or the layout differ from the profiled ones."""
import json
import os
import shutil

import bench


def test_kernel_bytes_of_the_large_lp():
    # 2e6 columns, 1e6 rows, 19,984,785 nonzeros, FP64: the per-launch figures
    # the bench line's roofline uses (matrix values and int32 columns, row
    # pointers, the gathered vector once, the epilogue's vectors)
    n, m, nnz = 2_000_000, 1_000_000, 19_984_785
    assert bench.kernel_bytes(0, n, m, nnz) == nnz * 12 + 4 * (m + 1) + 8 * n + 40 * m == 299_817_424
    assert bench.kernel_bytes(1, n, m, nnz) == nnz * 12 + 4 * (n + 1) + 8 * m + 80 * n + 48 * m == 463_817_424
    # FP32 values and vectors
    assert bench.kernel_bytes(0, n, m, nnz, s=4) == nnz * 8 + 4 * (m + 1) + 4 * n + 20 * m


def test_profiled_layout_reads_every_log_format(tmp_path):
    log = tmp_path / "stats.log"
    log.write_text("[bench] loaded in 1.1s (1.01 GiB on device), column slices (K, K') = (8, 4); layout K (S, "
                   "nnz/block, rows/block, split sums) = (8, 2048, 1024, 1), K' = (4, 1024, 256, 0)\n")
    assert bench.profiled_layout(str(tmp_path)) == {"K": [8, 2048, 1024, 1], "KT": [4, 1024, 256, 0]}
    log.write_text("[bench] column slices (K, K') = (8, 4); layout K (S, nnz/block, rows/block) = (8, 2048, 1024), "
                   "K' = (4, 2048, 1024)\n")
    assert bench.profiled_layout(str(tmp_path)) == {"K": [8, 2048, 1024], "KT": [4, 2048, 1024]}
    log.write_text("[bench] loaded, column slices (K, K') = (16, 2)\n")
    assert bench.profiled_layout(str(tmp_path)) == {"K": [16, 2048, 1024], "KT": [2, 2048, 1024]}
    log.write_text("nothing of the kind\n")
    assert bench.profiled_layout(str(tmp_path)) is None


def test_counter_traffic_needs_same_kernels_and_layout(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2312_14832_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("kernels.hip", "device.h", "internal.h"):
        shutil.copy(os.path.join(bench.ROOT, "paper_2312_14832_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    layout = {"K": [8, 2048, 1024, 1], "KT": [4, 2048, 1024, 1]}
    kern, wl = "k_partial_KT<double>+k_update<double>", "large_powerlaw_lp_n2000000"
    entry = {"source_sha": bench.kernel_source_sha(), "layout": layout, "traffic_bytes": 619.5e6}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({wl: {kern: entry}}))
    assert bench.counter_traffic(kern, wl, layout) == 619.5e6
    assert bench.counter_traffic(kern, wl, {"K": [8, 2048, 1024, 0], "KT": [4, 2048, 1024, 1]}) is None
    assert bench.counter_traffic(kern, "pagerank_lp_n1000000", layout) is None
    with open(csrc / "device.h", "a") as fh:   # any change to the kernel sources retires the counters
        fh.write("\n")
    assert bench.counter_traffic(kern, wl, layout) is None
