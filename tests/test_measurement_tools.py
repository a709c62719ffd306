"""Host-side measurement helpers (no GPU): the rocprofv3 counter summary and
the benchmark's rule for reporting counter traffic.

* traffic(): the median of a kernel's last working dispatches, scaled by what
  the same counter reads for the copy kernel of known size.
* bench_tiling(): the SpMV launch shape a benchmark run reported.
* measured_traffic(): the committed figure is reported only while the kernel
  sources and the launch shape match the ones the counters were taken with."""
import csv
import json
import os

import pytest

import bench
from paper_2510_08230_amd import profsum

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    spmv = "k_spmv_stream<double, EpiPq<double> >(long)"
    copy = "k_copy16(uint4 const*)"
    gib = 1 << 30
    # copy: 1 GiB read shows as 512 Ki KiB (scale 2), 1 GiB written as 1 Mi KiB (scale 1)
    fetch = [(copy, 524288.0)] + [(spmv, v) for v in (1.0, 900.0, 1000.0, 1100.0, 0.5)]
    write = [(copy, 1048576.0)] + [(spmv, v) for v in (0.2, 70.0, 80.0, 90.0, 0.1)]
    write_counters(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    write_counters(tmp_path / "w.csv", "WRITE_SIZE", write)
    d = profsum.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "EpiPq", gib, last=20)
    # launches reading under 1% of the largest returned at once and are dropped
    assert d["fetch_kib"] == 1000.0 and d["write_kib"] == 80.0
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    assert d["traffic_bytes"] == pytest.approx(1000.0 * 1024 * 2 + 80.0 * 1024)
    d2 = profsum.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "EpiPq", gib, last=1)
    assert d2["fetch_kib"] == 1100.0 and d2["write_kib"] == 90.0
    with pytest.raises(SystemExit):   # ambiguous name
        profsum.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_", gib)
    with pytest.raises(SystemExit):   # absent kernel
        profsum.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "EpiTrue", gib)


def tiling(remap=64, grid=1280):
    return {"spmv_kernel": 0, "lanes": 1, "grid": grid, "xcd_remap": remap, "exec_mode": 1, "chunk_iters": 0,
            "tuned": 1, "col_codes": 1, "spmv_ms": 0.18}


def test_bench_tiling_reads_the_json_line(tmp_path):
    log = tmp_path / "run.log"
    log.write_text("profiler noise\n" + json.dumps({"config": {"spmv_tiling": tiling(0, 1024)}}) + "\nmore noise\n")
    assert profsum.bench_tiling(str(log)) == {"spmv_kernel": 0, "lanes": 1, "grid": 1024, "xcd_remap": 0,
                                              "col_codes": 1}
    (tmp_path / "empty.log").write_text("no json here\n")
    with pytest.raises(SystemExit):
        profsum.bench_tiling(str(tmp_path / "empty.log"))


class Args:
    precision, seed, solver, precond, pattern, delta = "fp64", 1, "cg", "none", "stencil7", 1.0


def test_measured_traffic_needs_matching_sources_and_shape(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    rec = {"traffic_bytes": 1.2e9, "kernel_digest": profsum.kernel_digest(),
           "tiling": {k: tiling()[k] for k in profsum.TILING_KEYS}}
    (tmp_path / "profiles" / "spmv_pq_cg_fp64_stencil7_N215_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(Args, 215, tiling()) == 1.2e9
    assert bench.measured_traffic(Args, 215, tiling(remap=0)) is None     # another tile order
    assert bench.measured_traffic(Args, 215, tiling(grid=1024)) is None   # another grid
    assert bench.measured_traffic(Args, 100, tiling()) is None            # another workload
    other = Args()
    other.precision = "mixed_fp32"
    assert bench.measured_traffic(other, 215, tiling()) is None
    rec["kernel_digest"] = "0" * 16                                       # other kernel sources
    (tmp_path / "profiles" / "spmv_pq_cg_fp64_stencil7_N215_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic(Args, 215, tiling()) is None
