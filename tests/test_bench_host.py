"""Host-side logic of bench.py that needs no GPU: the traffic record built
from two counter passes, scaled by the calibration copy."""
import csv
import json
import os

import bench

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
        "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
        "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEAD)
        for k, (name, grid, val) in enumerate(rows):
            w.writerow([k, k, "Agent 1", 1, 1, 1, grid, 7, name, 512, 0, 0, 8, 0, 32, counter, val, 0, 1])


def test_traffic_record_scales_by_the_copy(tmp_path):
    n = bench.NPAIRS
    kern = f"void pdsink::{bench.PAIR_KERNEL_NAME}<7>(pdsink::PairParams)"
    fetch = [("__amd_rocclr_copyBuffer", 512, 3.0), (kern, n * 512, 1000.0),
             ("__amd_rocclr_copyBuffer", 131072, 131072.0)]   # the copy reads half its bytes per the counter
    write = [("__amd_rocclr_copyBuffer", 512, 1.0), (kern, n * 512, 10.0),
             ("__amd_rocclr_copyBuffer", 131072, 262144.0)]
    f, w, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _csv(f, "FETCH_SIZE", fetch)
    _csv(w, "WRITE_SIZE", write)
    bench.write_traffic(str(f), str(w), str(out))
    rec = json.load(open(out))
    assert rec["copy_calibration"]["fetch_factor"] == 2.0 and rec["copy_calibration"]["write_factor"] == 1.0
    assert rec["traffic_bytes"] == (1000.0 * 2.0 + 10.0) * 1024
    assert rec["source_hash"] == bench.source_hash()
    assert rec["algorithmic_bytes"] == n * (2 * 100 * 100 * 4 + 25)


def test_committed_traffic_record_is_for_these_sources():
    """The committed counter record is reported only while the pair kernel's
    sources hash to the value it was taken on."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "sinkhorn_fast_kernel_d100_1024pairs_traffic.json")
    rec = json.load(open(path))
    assert bench.measured_traffic() == (rec["traffic_bytes"] if rec["source_hash"] == bench.source_hash() else None)


def test_cpu_separable_stops_where_the_oracle_does():
    """bench.py's second CPU figure (K applied in the separable form of
    Proposition 2, log domain) runs Algorithm 1 as the dense oracle does: pair
    0 of the benchmark batch stops at tol 1e-3 at the iteration count the
    oracle wrote to the golden file."""
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sinkhorn_golden.json")
    stops = {c["index"]: c["iters"] for c in json.load(open(gold))["cases"] if c["kind"] == "stop_1e-3"}
    r = bench.cpu_separable(budget_s=300.0, n_pairs=1)
    assert r["iterations_to_tol"] == [stops[0]]
