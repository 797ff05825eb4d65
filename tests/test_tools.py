"""Host-side tools, no GPU: bench.py's command-line contract and the
rocprofv3 summary tool on small synthetic CSV files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        for r in rows:
            w.writerow(r)


def test_profile_summary_trace_and_traffic(tmp_path):
    from paper_1502_05216_amd import profile_summary as ps
    kern = "void (anonymous namespace)::k_twofold<double, 3, 2, 1>(double const*, double const*, " \
           "double*, double*, unsigned long)"
    copy = "__amd_rocclr_copyBuffer"
    hdr = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id",
           "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size",
           "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X",
           "Workgroup_Size_Y", "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    rows = []
    for i, dur in enumerate([900, 700, 600, 600, 620, 580]):
        rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 5, kern, i + 1, 1000 * i,
                     1000 * i + dur * 1000, 6144, 0, 52, 0, 106, 256, 1, 1, 786432, 1, 1])
    trace = tmp_path / "run_kernel_trace.csv"
    _write(trace, hdr, rows)
    out = tmp_path / "t.md"
    sys.argv = ["x", "trace", str(trace), "--title", "t", "--command", "c", "--select",
                "k_twofold<double", "--skip", "2", "--take", "3", "--out", str(out)]
    ps.main()
    text = out.read_text()
    assert "k_twofold<double,tlog1p> ept2 pd1" in text
    assert "| 3072 x 256 |" in text
    assert "606.7 (3..5)" in text           # mean of dispatches 3..5: (600 + 600 + 620) / 3
    # counters: a copy of n doubles reads FETCH n*8/2 KiB-units and writes n*8
    n = 1 << 20
    chdr = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
            "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    _write(fetch, chdr, [[1, 1, "Agent 1", 1, 1, 1, 1, 1, copy, 256, 0, 0, 8, 0, 8,
                          "FETCH_SIZE", n * 8 / 2 / 1024, 0, 1],
                         [2, 2, "Agent 1", 1, 1, 1, 1, 5, kern, 256, 0, 0, 8, 0, 8,
                          "FETCH_SIZE", n * 16 / 2 / 1024, 0, 1]])
    _write(write, chdr, [[1, 1, "Agent 1", 1, 1, 1, 1, 1, copy, 256, 0, 0, 8, 0, 8,
                          "WRITE_SIZE", n * 8 / 1024, 0, 1],
                         [2, 2, "Agent 1", 1, 1, 1, 1, 5, kern, 256, 0, 0, 8, 0, 8,
                          "WRITE_SIZE", n * 16 / 1024, 0, 1]])
    js = tmp_path / "traffic.json"
    sys.argv = ["x", "traffic", str(fetch), str(write), "--n", str(n), "--command-fetch", "f",
                "--command-write", "w", "--json", str(js), "--out", str(tmp_path / "tr.md")]
    ps.main()
    rec = json.load(open(js))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]["f64_tlog1p"]
    assert k["bytes_per_launch"] == pytest.approx(32 * n)
    assert k["algorithmic_bytes"] == 32 * n


def test_batch_candidates_are_valid_configurations():
    """Every autotuner candidate is a configuration the library accepts:
    an instantiated (ept64, ept32) pair, chunk_tiles in 1..4096, blocks per
    compute unit in 0..64 (tf_batch_plan_create's checks)."""
    from paper_1502_05216_amd import batch
    assert batch.DEFAULT_CONFIG in batch.CANDIDATES
    assert len(set(batch.CANDIDATES)) == len(batch.CANDIDATES) >= 12
    for e64, e32, ct, bpc in batch.CANDIDATES:
        assert (e64, e32) in ((2, 4), (4, 4), (1, 2))
        assert 1 <= ct <= 4096 and 0 <= bpc <= 64
