"""bench.py's command line on the CPU: it measures one GPU only and says so
for any other count, before touching a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--no-cpu-baseline", "--no-serve"):
        assert flag in r.stdout


def test_matrix_core_flops_follow_each_path_operands():
    # Per step, in units of 2*B*H*N*d^2.  bf16 applies S as hi + lo in the
    # apply (2); the fused query backward takes X = S G as hi + lo below
    # d = 128 and as the hi part at d = 128, plus the dS product; fp32
    # applies S as one operand everywhere.
    sys.path.insert(0, ROOT)
    import bench
    one = {"launches_per_step": 1.0}
    bf16_step = {k: one for k in ("summary_fwd", "apply", "bwd_query_ds", "bwd_key")}
    fp32_step = {k: one for k in ("summary_fwd", "apply", "bwd_query", "summary_bwd", "bwd_key")}
    unit = lambda d: 2 * d  # elems = 1
    assert bench.mma_flops_per_step(bf16_step, "bf16", 1, 128) == 7 * unit(128)
    assert bench.mma_flops_per_step(bf16_step, "bf16", 1, 64) == 8 * unit(64)
    assert bench.mma_flops_per_step(fp32_step, "fp32", 1, 128) == 6 * unit(128)
    # combine and the image builder do no products of the method
    assert bench.mma_flops_per_step({"combine": {"launches_per_step": 2.0}}, "bf16", 1, 128) == 0


def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


COUNTER_HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
                  "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
                  "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
                  "Counter_Value", "Start_Timestamp", "End_Timestamp"]
KEY = "void la::bwd_key_kernel<0, 0, 128, 3>(void const*, ...)"
COPY = "void (anonymous namespace)::stream_copy_swept_kernel<8, true>(...)"


def _counter_rows(counter, per_kernel):
    rows, i = [], 1
    for name, values in per_kernel:
        for v in values:
            rows.append([i, i, "Agent 1", 1, 1, 1, 1, 1, name, 256, 0, 0, 1, 0, 1, counter, v, 0, 1])
            i += 1
    return rows


def test_profile_summaries_from_rocprof_csv(tmp_path):
    # rocprofv3 output in the layout the GPU runs write: the summarizer
    # scales each kernel's mean counter per dispatch by the copy
    # calibration and records the current source digest
    import bench
    top = tmp_path / "prof"
    _write_csv(str(top / "trace" / "run_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"],
               [[KEY, 2, 6000000, 3000000.0, 90.0, 1, 1, 0], [COPY, 1, 600000, 600000.0, 10.0, 1, 1, 0]])
    _write_csv(str(top / "fetch" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("FETCH_SIZE", [(KEY, [100.0, 300.0])]))
    _write_csv(str(top / "write" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("WRITE_SIZE", [(KEY, [50.0, 50.0])]))
    # the calibration copy moves 1 GiB each way: FETCH_SIZE reads half of it
    _write_csv(str(top / "copy_fetch" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("FETCH_SIZE", [(COPY, [524288.0, 524288.0])]))
    _write_csv(str(top / "copy_write" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("WRITE_SIZE", [(COPY, [1048576.0])]))
    # the profiled runs' bench lines carry the digest of their sources
    for name in ("trace.out", "fetch.out", "write.out"):
        (top / name).write_text("log line\n" + json.dumps({"kernels": {}, "source_digest": bench.source_digest()}) + "\n")
    out = tmp_path / "profiles"
    out.mkdir()
    bench.summarize_profiles(str(top), str(out))
    rec = json.load(open(out / "counters_long_context_bf16.json"))
    assert rec["source_digest"] == bench.source_digest()
    assert rec["copy_factor_fetch"] == 2.0 and rec["copy_factor_write"] == 1.0
    k = rec["kernels"]["bwd_key"]
    assert k["fetch_kib"] == 200.0 and k["write_kib"] == 50.0 and k["dispatches"] == 2
    assert k["hbm_bytes_per_launch"] == (200.0 * 2 + 50.0) * 1024
    assert k["alg_bytes_per_launch"] == 4 * 8 * 2097152 * 128 * 2
    stats = open(out / "kernel_stats_long_context_bf16.txt").read()
    assert "bwd_key" in stats and "3000000" in stats
    # runs on other sources are refused a current digest
    (top / "write.out").write_text(json.dumps({"kernels": {}, "source_digest": "other"}) + "\n")
    import pytest
    with pytest.raises(SystemExit):
        bench.summarize_profiles(str(top), str(out))


def test_tiled_profile_summary_from_rocprof_csv(tmp_path):
    # the fused tiled step's summary: kernel statistics (the median launch
    # from the trace), counters scaled by the copy calibration, the field
    # passes of each kernel and the step's rate over the sum of medians
    import bench
    top = tmp_path / "prof"
    names = {"cols": "void la::(anonymous namespace)::tile_cols_kernel<64>(la::TGeo, ...)",
             "slots": "void la::(anonymous namespace)::tile_slot_kernel<64>(la::TGeo, ...)",
             "apply": "void la::(anonymous namespace)::tile_apply_kernel<64>(la::TGeo, ...)"}
    ms = {"cols": 2.0, "slots": 0.4, "apply": 2.4}
    _write_csv(str(top / "tiled_trace" / "run_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"],
               [[names[k], 3, ms[k] * 3e6, ms[k] * 1e6, 30.0, 1, 1, 0] for k in names])
    trace = []
    for k in names:
        for i, f in enumerate((1.5, 1.0, 1.0)):   # one slow first launch; median = ms[k]
            trace.append([names[k], 1000 * i, 1000 * i + int(ms[k] * f * 1e6)])
    _write_csv(str(top / "tiled_trace" / "run_kernel_trace.csv"),
               ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    _write_csv(str(top / "tiled_fetch" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("FETCH_SIZE", [(names["cols"], [4.0e6]), (names["apply"], [2.0e6])]))
    _write_csv(str(top / "tiled_write" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("WRITE_SIZE", [(names["cols"], [1.0e6]), (names["apply"], [4.0e6])]))
    _write_csv(str(top / "copy_fetch" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("FETCH_SIZE", [(COPY, [524288.0])]))
    _write_csv(str(top / "copy_write" / "run_counter_collection.csv"), COUNTER_HEADER,
               _counter_rows("WRITE_SIZE", [(COPY, [1048576.0])]))
    line = {"kernels_ms": {"tile_cols": 2.01, "tile_slots": 0.41, "tile_apply": 2.41},
            "tiled_source_digest": bench.source_digest(bench.TILED_SOURCES)}
    for name in ("tiled_trace.out", "tiled_fetch.out", "tiled_write.out"):
        (top / name).write_text(json.dumps(line) + "\n")
    out = tmp_path / "profiles"
    out.mkdir()
    bench.summarize_profiles(str(top), str(out))   # no long-context runs in DIR: tiled only
    text = open(out / "tiled_step_T256_Y64_X128_H16_d64.txt").read()
    field = 256 * 64 * 128 * 16 * 64 * 2
    rows = {l.split()[0]: l.split() for l in text.splitlines() if l.startswith("tile_")}
    assert rows["tile_cols"][3] == "2.0000"                         # median launch
    assert float(rows["tile_cols"][7]) == round((4.0e6 * 2 + 1.0e6) * 1024 / 1e9, 3)
    assert float(rows["tile_cols"][8]) == round(2 * field / 1e9, 3)
    assert rows["tile_slots"][9] == "-"                             # workspace only
    assert "step (sum of medians) 4.8000 ms" in text
    assert not (out / "counters_long_context_bf16.json").exists()
    # runs on other sources are refused
    (top / "tiled_write.out").write_text(json.dumps(dict(line, tiled_source_digest="other")) + "\n")
    import pytest
    with pytest.raises(SystemExit):
        bench.summarize_profiles(str(top), str(out))
