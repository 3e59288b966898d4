"""Host-side checks of the benchmark's measurement model (no GPU): the
algorithmic byte and flop counts per cell that bench.py divides by the
measured kernel times, checked against their definitions; the key that ties the committed
traffic counters to the kernel sources."""
import os

import bench


def test_bytes_per_cell():
    s = bench.STATE_BYTES
    assert s == 7 * 8
    # x-y pass (first, partial sum out): read the state, write the sum
    assert bench.sweep_bytes_per_cell(1, 0) == 2 * s
    # last pass of stage 1: state + running sum in, new state out
    assert bench.sweep_bytes_per_cell(0, 2) == 3 * s
    # stages 2 and 3 also read q^n
    assert bench.sweep_bytes_per_cell(0, 3) == 4 * s == bench.sweep_bytes_per_cell(0, 4)
    # float running sums (the FP32 form) are half as large
    assert bench.sweep_bytes_per_cell(0, 3, 28) == 3 * s + 28


def test_flops_per_cell():
    per_dir = bench.FLOPS_CONV + 7 * bench.FLOPS_WENO_VAR + bench.FLOPS_HLLC + bench.FLOPS_FLUXDIFF
    assert per_dir == 845
    assert bench.sweep_flops_per_cell(2, 0) == per_dir
    # the fused x-y pass converts each cell once for both directions
    assert bench.sweep_flops_per_cell(3, 0) == 2 * per_dir - bench.FLOPS_CONV
    # stage combinations: q_s + dt L (2 per variable), a q^n + b (q_s + dt L) (5)
    assert bench.sweep_flops_per_cell(2, 2) - per_dir == 7 * 2
    assert bench.sweep_flops_per_cell(2, 4) - per_dir == 7 * 5
    # WENO3 per variable: indicators 4, right edge 18, left 14
    assert bench.sweep_flops_per_cell(2, 0, 3) == per_dir - 7 * (97 - 36)


def test_ridge_selects_the_roof():
    ridge = bench.FP64_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
    xy = bench.sweep_flops_per_cell(3, 0) / bench.sweep_bytes_per_cell(1, 0)
    z = bench.sweep_flops_per_cell(2, 3) / bench.sweep_bytes_per_cell(0, 3)
    assert xy > ridge > z  # the x-y pass is compute-bound, the z pass memory-bound


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    import shutil

    import bench

    src = os.path.join(bench.ROOT, "paper_2409_10729_amd", "csrc")
    dst = tmp_path / "paper_2409_10729_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    f = dst / "physics.h"
    text = f.read_text()
    f.write_text("// a new comment\n/* and a\n   block */\n" + text.replace("{", "{ // brace", 1) + "\n\n")
    assert bench.source_hash() == h0
    f.write_text(text.replace("{", "{ int unused_marker = 0;", 1))
    assert bench.source_hash() != h0
    assert bench.code_of("a = 1; // c\n/* x\ny */ b = 2;\n\n") == "a = 1;\n b = 2;"
