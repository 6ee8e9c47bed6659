"""bench.py's command line on the CPU: more than one GPU is refused before
anything touches a GPU (this build measures one GPU; sharding is designed,
not built)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields(inputs):
    """The oracle leg of the benchmark on a tiny workload: single-thread walk
    and index, all-thread queries, with the CPU model and thread counts."""
    sys.path.insert(0, ROOT)
    import bench

    g = inputs.ba_graph(1000, 5)
    q = inputs.queries_uniform(g, 16, 101, over="all")
    cb = bench.cpu_baseline(g, q, 5, 10, 1, 20_000)
    assert cb["kind"] == "oracle" and cb["unit"] == "path-steps/s" and cb["value"] > 0
    assert cb["cores"] >= 1 and cb["nproc"] >= 1 and cb["cpu_model"]
    assert cb["single_thread"]["walk_path_steps_per_s"] > 0
    assert cb["all_threads"]["queries_per_s"] > 0


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench

    # index: 4 B per path vertex read, 4 B per entry written, 8 B per offset
    assert bench.index_algorithmic_bytes(10, 5, 50, 7) == 4 * 60 + 4 * 50 + 8 * 8
    # count: 16 B per query, 28 B per listed path, 8 B per output slot
    assert bench.count_algorithmic_bytes(np.array([3, 0, 5]), 2) == 16 * 3 + 28 * 8 + 8 * 2 * 3
