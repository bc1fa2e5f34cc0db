"""bench.py command line on the CPU: more than one GPU is refused with a
message before anything touches a device."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_record_is_dropped_when_the_loop_source_changes(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "_loop_source_hash", lambda workload, prec: "0" * 64)
    assert bench._traffic("rashba_s9_L24", "fp32") is None


def test_flop_counts_of_the_loop():
    """Survey count of the six-orbital loop per (q, k, channel): separable ky
    transform over 9 phases, halved by hermiticity, plus the block build
    (8 n_o^2 n_b (n_b + n_o^2)); matrix-core flops of the real-basis kernel:
    21 row tiles x 36 columns x 6 bands x 2, three BF16 products."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.credited_loop_flops_per_pair(6, 4) == 8 * 9 * 1296 // 2 + 8 * 36 * 6 * 42 == 119232
    assert bench.mfma_flops_per_pair(4) == 3 * 2 * 336 * 36 * 6
    assert bench.mfma_flops_per_pair(2) == 3 * 2 * 192 * 36 * 6
    # Kramers pairs: three bands summed
    assert bench.mfma_flops_per_pair(4, 6, 3) == 3 * 2 * 336 * 36 * 3
    assert bench.credited_loop_flops_per_pair(6, 4, 3) == 8 * 9 * 1296 // 2 + 8 * 36 * 3 * 39 == 80352
    model, n = bench._cpu_info()
    assert isinstance(model, str) and n >= 1


def _counter_csv(path, rows):
    head = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
            '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
            '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"')
    with open(path, "w") as fh:
        fh.write(head + "\n")
        for d, name, counter, v in rows:
            fh.write(f'{d},{d},"Agent 1",1,1,1,512,8,"{name}",512,0,0,8,0,32,"{counter}",{v},0,1\n')


def test_traffic_summary_from_counter_csvs(tmp_path, monkeypatch):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of the loop kernel (other kernels
    ignored), scaled per byte by the largest three copy dispatches."""
    sys.path.insert(0, ROOT)
    import argparse

    import bench
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_loop_source_hash", lambda workload, prec: "ab" * 32)
    dirs = [tmp_path / n for n in ("f", "w", "cf", "cw")]
    for d in dirs:
        d.mkdir()
    k = "void tufrg::loop_rb_kernel<4, 0>(float const*)"
    _counter_csv(dirs[0] / "fetch_counter_collection.csv",
                 [(1, k, "FETCH_SIZE", 100.0), (2, "other", "FETCH_SIZE", 5e9), (3, k, "FETCH_SIZE", 300.0)])
    _counter_csv(dirs[1] / "write_counter_collection.csv", [(1, k, "WRITE_SIZE", 40.0), (3, k, "WRITE_SIZE", 60.0)])
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(dirs[2] / "fetch_counter_collection.csv",
                 [(1, copy, "FETCH_SIZE", 1.0), (2, copy, "FETCH_SIZE", 2 ** 19), (3, copy, "FETCH_SIZE", 2 ** 19),
                  (4, copy, "FETCH_SIZE", 2 ** 19)])
    _counter_csv(dirs[3] / "write_counter_collection.csv",
                 [(2, copy, "WRITE_SIZE", 2 ** 20), (3, copy, "WRITE_SIZE", 2 ** 20), (4, copy, "WRITE_SIZE", 2 ** 20)])
    args = argparse.Namespace(summarize_traffic=[str(d) for d in dirs], workload="t2g_s13_L48", prec="bf16x3")
    bench.summarize_traffic(args)
    import json
    t = json.load(open(tmp_path / "profiles" / "loop_kernel_traffic_t2g_s13_L48_bf16x3.json"))
    assert t["dispatches"] == 2 and t["fetch_kib_per_dispatch"] == 200.0 and t["write_kib_per_dispatch"] == 50.0
    assert t["copy_calibration"]["fetch_bytes_per_kib"] == 2048.0 and t["copy_calibration"]["write_bytes_per_kib"] == 1024.0
    assert t["hbm_bytes_per_launch"] == 200.0 * 2048 + 50.0 * 1024
    assert bench._traffic("t2g_s13_L48", "bf16x3") == t["hbm_bytes_per_launch"]


def test_trace_summary_from_kernel_stats(tmp_path):
    sys.path.insert(0, ROOT)
    import argparse

    import bench
    p = tmp_path / "kt_kernel_stats.csv"
    p.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
                 '"small",10,1000,100,10.0,90,110,1\n"big",2,9000,4500,90.0,4000,5000,10\n')
    out = tmp_path / "s.md"
    bench.summarize_trace(argparse.Namespace(summarize_trace=[str(p), "rocprofv3 ... -- python3 bench.py", str(out)],
                                             workload="w", prec="bf16x3"))
    text = out.read_text().splitlines()
    rows = [r for r in text if r.startswith("| `")]
    assert rows[0].startswith("| `big` | 2 | 0.009 | 4.5") and "90.0 %" in rows[0]
    assert "rocprofv3 ... -- python3 bench.py" in text


def test_counter_summary_per_dispatch_and_per_wave_tile(tmp_path):
    """SQ counters of the loop kernel summed per dispatch (other kernels
    ignored) and divided per wave and ky tile: 48 x 16 / 16 = 48 tiles per
    wave on the 48 x 48 mesh refined 16x."""
    sys.path.insert(0, ROOT)
    import argparse

    import bench
    k = "void tufrg::loop_rb_kernel<4, 0>(float const*)"
    rows = []
    for d in (1, 2):
        rows += [(d, k, "SQ_WAVES", 100), (d, k, "SQ_INSTS_VALU", 100 * 48 * 500),
                 (d, k, "SQ_INSTS_MFMA", 100 * 48 * 200), (d, k, "SQ_INSTS_LDS", 100 * 48 * 50),
                 (d, k, "SQ_LDS_BANK_CONFLICT", 100 * 48 * 25), (d, "other_kernel", "SQ_WAVES", 7)]
    _counter_csv(tmp_path / "sq.csv", rows)
    out = tmp_path / "sq.md"
    args = argparse.Namespace(summarize_counters=[str(tmp_path / "sq.csv"), "rocprofv3 --pmc ...", str(out)],
                              workload="t2g_s13_L48", prec="bf16x3", six_bands=True)
    bench.summarize_counters(args)
    text = out.read_text()
    assert "2 dispatches" in text and "| SQ_WAVES | 100 |" in text and "rocprofv3 --pmc ..." in text
    assert "SQ_INSTS_VALU: 500" in text and "SQ_INSTS_MFMA: 200" in text and "SQ_INSTS_LDS: 50" in text
    assert "per LDS instruction: 0.50" in text
    # the same counters as a paired run: 384 ky pairs per row, 24 tiles
    args.six_bands = False
    bench.summarize_counters(args)
    text = out.read_text()
    assert "16 ky pairs" in text and "SQ_INSTS_VALU: 1000" in text


def test_source_hash_ignores_comments_and_layout():
    sys.path.insert(0, ROOT)
    import bench
    a = "int f(int x) {  // twice\n  return 2 * x; /* doubled */\n}\n"
    b = "int f(int x) {\n    return 2 * x;\n}"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(b.replace("2 *", "3 *"))
