"""Host-side checks of the benchmark script (no GPU needed)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_defines_its_legs():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("main", "run_single", "fp64_beside", "chain_roofline", "served_block", "cpu_baseline",
                 "host_description", "bench_batched", "bench_dmc", "bench_served", "copy_reference"):
        assert callable(getattr(bench, name)), name
    host = bench.host_description()
    assert host["nproc"] >= 1 and host["affinity_cpus"] >= 1


def test_bench_refuses_several_gpus(capsys):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_traffic_records_are_consistent():
    """Each committed HBM-traffic record (rocprofv3 FETCH_SIZE / WRITE_SIZE per dispatch, scaled by
    a plain copy's readings) names existing sources and adds up: traffic = fetch x factor + write x
    factor, in bytes, with the factors those of the copy calibration."""
    import glob
    import json
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic_*.json")))
    assert paths
    for p in paths:
        d = json.load(open(p))
        for f in d["source_files"]:
            assert os.path.exists(os.path.join(ROOT, f)), (p, f)
        c = d["copy_calibration"]
        assert abs(d["fetch_factor"] - c["bytes_read_and_written"] / (c["fetch_size_kib"] * 1024.0)) < 1e-9
        assert abs(d["write_factor"] - c["bytes_read_and_written"] / (c["write_size_kib"] * 1024.0)) < 1e-9
        t = 1024.0 * (d["fetch_size_kib_per_dispatch"] * d["fetch_factor"] +
                      d["write_size_kib_per_dispatch"] * d["write_factor"])
        assert abs(d["traffic_bytes_per_dispatch"] - t) <= 1e-9 * t, p


def test_traffic_record_is_dropped_once_its_sources_change(tmp_path, monkeypatch):
    """measured_traffic returns a record's bytes while the hash of the sources it names matches,
    and None once they change (or for a kernel with no record)."""
    import json
    import types
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "kernel.hip"
    src.write_text("// version 1\n")
    rec = {"source_files": ["kernel.hip"], "source_sha256_16": bench.source_hash(["kernel.hip"]),
           "traffic_bytes_per_dispatch": 1234.0}
    (tmp_path / "profiles" / "chain_traffic_toy.json").write_text(json.dumps(rec))
    wl = types.SimpleNamespace(name="toy")
    assert bench.measured_traffic(wl, "chain") == 1234.0
    assert bench.measured_traffic(wl) is None            # no gather record
    src.write_text("// version 2\n")
    assert bench.measured_traffic(wl, "chain") is None
