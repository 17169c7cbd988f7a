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


def test_profile_summaries_from_rocprof_csv(tmp_path, capsys):
    """The profile summaries bench.py writes from rocprofv3 CSV files: the
    kernel-trace summary leaves out the warm-up dispatches of each kernel,
    and the traffic summary scales the counters by the copy calibration."""
    sys.path.insert(0, ROOT)
    import json
    import bench
    trace = tmp_path / "kt.csv"
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp"]
    name = "void falcon_dev::k_decompress<falcon_dev::TF64>(falcon_dev::DecompressArgs)"
    for i, d in enumerate([5000, 1000, 1002, 998]):  # one slow warm-up dispatch, then 3 timed
        rows.append(f'"{name}",{i * 10000},{i * 10000 + d * 1000}')
    trace.write_text("\n".join(rows) + "\n")
    got = bench.trace_summary(str(trace), 1)
    assert abs(got["k_decompress"] - 1000.0) < 1e-9
    fetch, write, bj = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "b.json"
    hdr = "Kernel_Name,Counter_Name,Counter_Value"
    fetch.write_text(hdr + "\n__amd_rocclr_copyBuffer,FETCH_SIZE,512\n" + f'"{name}",FETCH_SIZE,300\n')
    write.write_text(hdr + "\n__amd_rocclr_copyBuffer,WRITE_SIZE,1024\n" + f'"{name}",WRITE_SIZE,1024\n')
    bj.write_text(json.dumps({"config": {"bytes": 1 << 20, "workload": "w"},
                              "kernel_algorithmic_bytes": {"k_decompress": 1400 * 1024}}) + "\n")
    rec = bench.traffic_summary(str(fetch), str(write), str(bj))
    k = rec["kernels"]["k_decompress"]
    # copy of 1 MiB: FETCH_SIZE reads half (factor 2), WRITE_SIZE all (factor 1)
    assert k["hbm_bytes_per_launch"] == 300 * 1024 * 2 + 1024 * 1024
    capsys.readouterr()
