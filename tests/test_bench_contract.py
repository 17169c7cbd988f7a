"""bench.py keeps its command-line contract without a GPU: every section it
runs exists, and more than one GPU is refused with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sections_exist():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("cpu_baseline", "host_pipeline", "batched", "serving", "ablation", "float32_case", "oracle_small_case", "studies", "full_range", "measured_traffic",
                 "kernel_source_digest", "main"):
        assert callable(getattr(bench, name)), name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
