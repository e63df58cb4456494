"""The benchmark's command line (no GPU needed): more than one GPU is
refused with a message, and the oracle baseline runs on a tiny sample."""
import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_baseline_reports_single_and_threaded_oracle():
    import bench
    args = types.SimpleNamespace(cpu_sample_shards=2, data_seed=7, b=8, seed=0,
                                 workload="vfilter")
    cb = bench.cpu_baseline(args)
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == "Mkeys/s"
    assert cb["value"] > 0 and cb["query_value"] > 0
    par = cb["parallel"]
    assert 1 <= par["threads"] <= 16 and par["value"] > 0 and par["query_value"] > 0
