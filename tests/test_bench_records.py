"""bench.py's command-line contract and the counter records it reads, on the
CPU: the committed HBM-traffic records must have been taken on the kernel
sources in the tree (else the bench line reports null traffic), and the
benchmark refuses more than one GPU with a message."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    import importlib
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        return importlib.import_module("bench")
    finally:
        sys.argv = argv


def test_traffic_records_match_the_kernel_sources():
    b = _bench()
    t = b.measured_traffic()
    assert t is not None and t > 0, "profiles/k_rmd_persistent_traffic.json was taken on other sources"
    s = b.measured_scps_traffic()
    assert s is not None, "profiles/k_scps_traffic_chain6000x32.json was taken on other sources"
    # the stack is read once per pass (51 frames x 17,997,000 pairs x 4 B); the
    # counters cannot show less than that
    stack = 51 * 17_997_000 * 4
    assert s["distance"] >= stack and s["bias"] >= stack
    with open(os.path.join(ROOT, "profiles", "k_scps_traffic_chain6000x32.json")) as f:
        rec = json.load(f)
    assert all("rocprofv3 --pmc" in c for c in rec["commands"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
