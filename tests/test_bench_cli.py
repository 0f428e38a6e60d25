"""Host-side checks of the benchmark script (no GPU): the one-GPU contract
for --gpus, and the consistency of its workload tables."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_tables_are_consistent():
    import bench
    for table in (bench.WALLS, bench.CURVED, bench.MODEL_CS):
        assert set(table) <= set(bench.WORKLOADS)
    for name, spec in bench.WORKLOADS.items():
        N, nelem, eq, vf, sf, mu, blend, desc = spec
        assert 1 <= N <= 7 and len(nelem) == 3 and eq in (0, 1) and blend in (0, 1) and desc
        assert (eq == 1) == (mu > 0.0), name
        if name in bench.WALLS or name in bench.MODEL_CS:
            assert eq == 1, name
    assert bench.WORKLOADS["tgv_n5_32"][1] == (32, 32, 32)
    assert bench.WORKLOADS["tgv_n7_64"][:2] == (7, (64, 64, 64))
    traffic = {k for k in bench.MEASURED_TRAFFIC if k != "kernel_sha"}
    assert traffic <= set(bench.WORKLOADS)
    for k in traffic:
        t = bench.MEASURED_TRAFFIC[k]
        assert abs(t["fetch"] + t["write"] - t["bytes_per_launch"]) <= 1e-3 * t["bytes_per_launch"], k


def test_counters_and_profiles_match_the_kernel_source():
    """The HBM traffic and FP64 counts bench.py reports were collected on the
    kernel source in the tree (else it reports traffic null), and the
    rocprofv3 summaries of the headline workload name the same source."""
    import bench
    sha = bench.kernel_sha()
    assert bench.MEASURED_TRAFFIC["kernel_sha"] == sha, "kernel changed since the counters were taken"
    for f in ("k_stage_tgv_n7_64.md", "k_stage_tgv_n5_32.md"):
        with open(os.path.join(ROOT, "profiles", f)) as fh:
            assert sha in fh.read(), f
