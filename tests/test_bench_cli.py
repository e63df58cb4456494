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


def test_cpu_baseline_reports_threaded_and_single_thread_oracle():
    import bench
    args = types.SimpleNamespace(cpu_sample_shards=2, data_seed=7, b=8, seed=0,
                                 workload="vfilter", log2n=17, eps=0.08)
    cb = bench.cpu_baseline(args)
    assert cb["kind"] == "oracle" and cb["unit"] == "Mkeys/s"
    assert 1 <= cb["cores"] <= 16 and cb["value"] > 0 and cb["query_value"] > 0
    one = cb["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0 and one["query_value"] > 0
