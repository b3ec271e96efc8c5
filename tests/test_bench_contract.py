"""The benchmark script's host-side contract: a run on more than one GPU is refused with a
message, and the stored HBM-traffic figure and its profile summary name the same kernel
source and byte count."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_matches_its_profile_summary():
    sys.path.insert(0, ROOT)
    import bench
    for (kernel, workload), m in bench.MEASURED_TRAFFIC.items():
        text = open(os.path.join(ROOT, m["summary"])).read()
        assert kernel in text and workload in text
        sha = re.search(r"sha256 ([0-9a-f]{16})", text).group(1)
        assert sha == m["sha256_16"]
        mb = float(re.search(r"Per step \(.*?\): ([0-9.]+) MB measured", text).group(1))
        assert abs(mb * 1e6 - m["bytes_per_step"]) < 0.06e6
