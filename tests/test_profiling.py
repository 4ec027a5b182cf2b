"""Host-side: the rocprofv3 summaries used for the traffic figure."""
import csv

from paper_1802_06922_amd import profiling


def _pmc(path, rows):
    """rows: (kernel, counter, value) or (kernel, counter, value, grid size); dispatch ids in order."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for d, row in enumerate(rows):
            k, c, v = row[:3]
            grid = row[3] if len(row) > 3 else 1024
            w.writerow({"Dispatch_Id": d + 1, "Grid_Size": grid, "Kernel_Name": k, "Counter_Name": c,
                        "Counter_Value": v})


def test_traffic_record_scales_by_the_copy(tmp_path):
    g = "void qmc::k_gather<double>(qmc::SysParams, ...)"
    # two initialisation launches of another shape (ignored), then the timed launches
    _pmc(tmp_path / "f.csv", [(g, "FETCH_SIZE", 9000.0, 2048), (g, "FETCH_SIZE", 7.0, 2048),
                              (g, "FETCH_SIZE", 1000.0), (g, "FETCH_SIZE", 1200.0),
                              ("qmc::k_chain", "FETCH_SIZE", 5.0)])
    _pmc(tmp_path / "w.csv", [(g, "WRITE_SIZE", 50.0, 2048), (g, "WRITE_SIZE", 300.0)])
    copy = 1 << 30
    # a copy whose FETCH_SIZE reads half the bytes moved and whose WRITE_SIZE reads all of them
    _pmc(tmp_path / "cf.csv", [("elementwise_copy", "FETCH_SIZE", copy / 2048.0)] * 3)
    _pmc(tmp_path / "cw.csv", [("elementwise_copy", "WRITE_SIZE", copy / 1024.0)] * 3)
    d = profiling.traffic_json("w", "k_gather<double>", str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                               str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv"), copy, ["cmd"])
    assert abs(d["fetch_factor"] - 2.0) < 1e-12 and abs(d["write_factor"] - 1.0) < 1e-12
    assert d["fetch_size_kib_per_dispatch"] == 1100.0
    assert abs(d["traffic_bytes_per_dispatch"] - (1100.0 * 1024 * 2 + 300.0 * 1024)) < 1e-6
    assert d["source_sha256_16"] == profiling.source_hash(profiling.GATHER_SOURCES)


def test_stats_markdown(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "void qmc::k_gather<double>(int)", "Calls": 3, "AverageNs": 2500.0,
                    "MinNs": 2000.0, "MaxNs": 3000.0, "Percentage": 50.0})
    md = profiling.stats_md(str(p), "t", "cmd")
    assert "| `qmc::k_gather<double>` | 3 | 2.5 | 2.0 | 3.0 | 50.0% |" in md
