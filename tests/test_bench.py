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
