"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message, and the committed HBM-counter record it reports as
`traffic` is tied to the current source of the swept kernel."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_matches_kernel_source():
    sys.path.insert(0, ROOT)
    import bench
    rec = None
    for line in open(os.path.join(ROOT, "profiles", "k_dense_sweep_n30_c64_hbm_counters.md")):
        if line.startswith("traffic-record:"):
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
    assert rec is not None
    src = open(os.path.join(ROOT, rec["src"]), "rb").read()
    if hashlib.sha256(src).hexdigest() == rec["src_sha256"]:
        # the sweep moves each amplitude once: 8 B read + 8 B written at n = 30
        assert abs(bench.recorded_traffic() / (16.0 * (1 << 30)) - 1.0) < 0.01
    else:
        assert bench.recorded_traffic() is None
