"""CPU: the rocprofv3 summary tool on small synthetic CSV files (per-dispatch
means, the copy calibration, bytes by TCC request size, the counters'
derived rates)."""
import csv
import json

import pytest

from paper_2208_08038_amd import profile_summary as ps

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow({k: r.get(k, 0) for k in FIELDS})


def _rows(kernel, counter, values, grid=1024, t0=0, dur=1000, instances=2):
    """One row per (dispatch, counter instance); the instances of a
    dispatch sum to the value."""
    out = []
    for d, v in enumerate(values):
        for i in range(instances):
            out.append({"Dispatch_Id": d + 1, "Kernel_Name": kernel, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": v / instances,
                        "Start_Timestamp": t0 + 10 * dur * d,
                        "End_Timestamp": t0 + 10 * dur * d + dur})
    return out


def test_traffic_scales_by_the_copy_and_counts_request_sizes(tmp_path):
    K, C = "k_push_tiled_f32<3, true, 2, 4, 8, 8, 6>(args)", "__amd_rocclr_copyBuffer"
    copy_bytes = 2.0 ** 31
    f = tmp_path
    _write(f / "fk.csv", _rows(K, "FETCH_SIZE", [1000.0, 1200.0]))
    _write(f / "wk.csv", _rows(K, "WRITE_SIZE", [500.0, 500.0]))
    # the copy fetches half of what it moves by this counter; a small copy
    # of another grid size is left out
    _write(f / "fc.csv", _rows(C, "FETCH_SIZE", [copy_bytes / 2048.0] * 3, grid=4096) +
           _rows(C, "FETCH_SIZE", [7.0], grid=64))
    _write(f / "wc.csv", _rows(C, "WRITE_SIZE", [copy_bytes / 1024.0] * 3, grid=4096))
    # request counts: reads 128 B and 64 B, writes 64 B and 32 B
    t1 = (_rows(K, "TCC_EA0_RDREQ_32B_sum", [0, 0]) + _rows(K, "TCC_EA0_RDREQ_64B_sum", [10, 10]) +
          _rows(K, "TCC_EA0_RDREQ_128B_sum", [100, 100]))
    t2 = _rows(K, "TCC_EA0_WRREQ_sum", [50, 50]) + _rows(K, "TCC_EA0_WRREQ_64B_sum", [40, 40])
    t1c = _rows(C, "TCC_EA0_RDREQ_32B_sum", [0], grid=4096) + \
        _rows(C, "TCC_EA0_RDREQ_64B_sum", [0], grid=4096) + \
        _rows(C, "TCC_EA0_RDREQ_128B_sum", [copy_bytes / 128], grid=4096)
    t2c = _rows(C, "TCC_EA0_WRREQ_sum", [copy_bytes / 64], grid=4096) + \
        _rows(C, "TCC_EA0_WRREQ_64B_sum", [copy_bytes / 64], grid=4096)
    for name, rows in (("t1.csv", t1), ("t2.csv", t2), ("t1c.csv", t1c), ("t2c.csv", t2c)):
        _write(f / name, rows)

    class A:
        pass

    a = A()
    a.fetch, a.write, a.copy_fetch, a.copy_write = (str(f / n) for n in
                                                    ("fk.csv", "wk.csv", "fc.csv", "wc.csv"))
    a.copy_bytes, a.copy_kernel, a.kernel, a.workload = copy_bytes, C, K[:-6], "w"
    a.command, a.out = ["cmd"], str(f / "t.json")
    a.req_read, a.req_write = str(f / "t1.csv"), str(f / "t2.csv")
    a.req_copy_read, a.req_copy_write = str(f / "t1c.csv"), str(f / "t2c.csv")
    ps.traffic(a)
    t = json.load(open(a.out))
    assert t["scale_fetch"] == pytest.approx(2.0) and t["scale_write"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(1100.0 * 1024 * 2.0)
    assert t["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert t["by_request_size"]["read_bytes"] == pytest.approx(64 * 10 + 128 * 100)
    assert t["by_request_size"]["write_bytes"] == pytest.approx(64 * 40 + 32 * 10)
    assert t["by_request_size_copy"]["read_bytes"] == pytest.approx(copy_bytes)
    assert t["by_request_size_copy"]["write_bytes"] == pytest.approx(copy_bytes)
    assert t["kernel_source_hash"] == ps.kernel_source_hash()


def test_counters_derive_issue_rate_and_per_pair_counts(tmp_path):
    K = "k_push_tiled_f32<3, true, 2, 4, 8, 8, 6>(args)"
    dur_ns = 400_000  # 400 us per dispatch
    valu = 0.5 * dur_ns * 1e-9 * 2.4e9 * 256  # half of one wave instruction per CU per clock
    _write(tmp_path / "a.csv", _rows(K, "SQ_INSTS_VALU", [valu, valu], dur=dur_ns) +
           _rows(K, "SQ_INSTS_LDS", [640.0, 640.0], dur=dur_ns))
    _write(tmp_path / "b.csv", _rows(K, "SQ_INSTS_VALU_FMA_F32", [64.0, 64.0], dur=dur_ns) +
           _rows(K, "SQ_LDS_BANK_CONFLICT", [30.0, 30.0], dur=dur_ns) +
           _rows(K, "SQ_ACTIVE_INST_LDS", [20.0, 20.0], dur=dur_ns))

    class A:
        pass

    a = A()
    a.csv = [str(tmp_path / "a.csv"), str(tmp_path / "b.csv")]
    a.kernel, a.pairs, a.clock, a.cus = "k_push_tiled_f32<3, true, 2", 64.0, 2.4e9, 256
    a.title, a.command, a.note, a.out = "t", ["cmd"], None, str(tmp_path / "c.txt")
    ps.counters(a)
    text = open(a.out).read()
    vals = {}
    for line in text.splitlines():
        parts = line.split()
        if parts and parts[-1].replace(".", "", 1).isdigit():
            vals[" ".join(parts[:-1])] = float(parts[-1])
    assert vals["VALU issue (one wave instruction per CU per clock)"] == pytest.approx(0.5)
    assert vals["LDS per pair"] == pytest.approx(640.0)
    assert vals["FP32 FMA+MUL+ADD per pair"] == pytest.approx(64.0)
    assert vals["LDS bank-conflict / LDS-active cycles"] == pytest.approx(1.5)
    assert f"# kernel source hash: {ps.kernel_source_hash()}" in text
