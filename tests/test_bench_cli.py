"""CPU checks of the benchmark script's host logic: the one-GPU guard, the
kernel-trace and sweep-segment summaries on hand-made traces, the kernel
names of the tile shapes and the counter bookkeeping.  No GPU needed."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for name, grid, dur in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 100


def test_trace_summary_groups_by_kernel_and_grid(tmp_path, capsys):
    p = tmp_path / "k.csv"
    _trace(p, [("void a<1>(int)", 64, 1000), ("void a<1>(int)", 64, 3000), ("void a<1>(int)", 128, 500),
               ("void b(int)", 64, 10000)])
    bench.trace_summary(str(p))
    out = capsys.readouterr().out.splitlines()
    assert out[2].startswith("| `b` | 64 | 1 | 10.00 |")
    assert out[3].startswith("| `a<1>` | 64 | 2 | 2.00 | 1.00 | 3.00 | 0.004 |")
    assert out[4].startswith("| `a<1>` | 128 | 1 | 0.50 |")


def test_segment_summary_splits_a_sweep_into_its_segments(tmp_path, capsys):
    # a sweep of N = 4 slots: prologue, 3 x (phase 1, phase 2), stopping rule
    N = 4
    rows = [("void rpr::k_sweep_pass<3>(int)", 1024, 5000)] * 3
    seg = "void rpr::k_chain_seg<3, float>(int)"
    rows += [(seg, 1024, 7000)] + [(seg, 1024, d) for _ in range(N - 1) for d in (2000, 4000)] + [(seg, 1024, 9000)]
    p = tmp_path / "s.csv"
    _trace(p, rows)
    bench.segment_summary(str(p), N=N)
    out = capsys.readouterr().out
    assert "| 1 | `rpr::k_chain_seg<3, float>` | 7.0 | 2.00 / 2.00 | 4.00 / 4.00 | 9.0 | 0.03 |" in out
    assert "3 dispatches, mean 5.00 us" in out


@pytest.mark.parametrize("shape,real,name", [("R5NW8", "float", "k_prop_swe_fused<float, 5, 8>"),
                                             ("rows:C3R2NW12", "float", "k_prop_swe_rows<float, 3, 2, 12>"),
                                             ("R4NW8", "double", "k_prop_swe_fused<double, 4, 8>")])
def test_kernel_names_of_tile_shapes(shape, real, name):
    assert bench.swe_kernel_name(shape, real) == name


def test_traffic_only_for_the_sources_and_shape_the_counters_were_taken_on(monkeypatch):
    h = bench.sources_hash(bench.PROP_SOURCES)
    t = {"sources": h, "fetch_scale": 2.0, "write_scale": 1.0, "shapes": {"R5NW8": (100.0, 200.0)}}
    monkeypatch.setattr(bench, "PROP_TRAFFIC", t)
    assert bench.measured_traffic("R5NW8") == (100.0 * 2.0 + 200.0) * 1024
    assert bench.measured_traffic("R4NW8") is None
    monkeypatch.setattr(bench, "PROP_TRAFFIC", dict(t, sources="0" * 16))
    assert bench.measured_traffic("R5NW8") is None


def test_trace_window_takes_the_dispatches_of_one_solve(tmp_path, capsys):
    import json
    rows = [("void k<float, 5, 8>(int)", 96, d) for d in (1, 2, 3, 4, 5, 6)] + [("void k<float, 5, 8>(int)", 48, 100)]
    p = tmp_path / "w.csv"
    _trace(p, rows)
    bench.trace_window(str(p), "k<float, 5, 8>", 96, 1, 3)
    out = json.loads(capsys.readouterr().out)
    assert out["dispatches"] == 6 and out["window"] == [2, 5]
    assert abs(out["mean_us"] - 0.004) < 1e-12
